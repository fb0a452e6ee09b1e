"""Reference restricted Hartree-Fock iterations for the SCF tests (TEST INFRASTRUCTURE): numpy
linear algebra with the oracle's one-electron integrals and J/K. Roothaan iterations from the
core-Hamiltonian guess, optionally with Pulay's DIIS on the commutator FDS - SDF and a level
shift of the virtual orbitals."""
import numpy as np

import oracle


def rhf(mol, charges, niter=10, diis=0, tau=None, level_shift=0.0):
    o = oracle.Oracle(mol)
    S, T, V, enuc = o.one_electron(charges)
    H = T + V
    nocc = int(round(np.sum(charges))) // 2
    s, U = np.linalg.eigh(S)
    keep = s > 1e-8 * s.max()
    X = U[:, keep] / np.sqrt(s[keep])

    def density(F):
        e, Cp = np.linalg.eigh(X.T @ F @ X)
        C = X @ Cp[:, :nocc]
        return 2.0 * C @ C.T

    D = density(H)
    energies = []
    fs, es = [], []
    for _ in range(niter):
        J, K = o.jk(D=D, tau=mol.thresh if tau is None else tau)
        F = H + J - 0.5 * K
        energies.append(0.5 * np.sum(D * (H + F)) + enuc)
        if diis:
            err = X.T @ (F @ D @ S - S @ D @ F) @ X
            fs.append(F)
            es.append(err)
            fs, es = fs[-diis:], es[-diis:]
            n = len(fs)
            B = -np.ones((n + 1, n + 1))
            B[n, n] = 0.0
            for i in range(n):
                for j in range(n):
                    B[i, j] = np.sum(es[i] * es[j])
            rhs = np.zeros(n + 1)
            rhs[n] = -1.0
            c = np.linalg.solve(B, rhs)
            F = sum(ci * fi for ci, fi in zip(c[:n], fs))
        if level_shift:
            F = F + level_shift * (S - 0.5 * S @ D @ S)
        D = density(F)
    return np.array(energies)
