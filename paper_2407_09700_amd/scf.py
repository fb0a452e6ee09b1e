"""Restricted Hartree-Fock iterations around the J/K build.

The workload of the paper's SCF benchmarks (section 5, Table 1): Roothaan iterations whose Fock
matrix F = H + J - K/2 takes J and K from the integral-direct build, with one plan (shell pairs,
Schwarz factors, work-list layout) made once and reused by every iteration. The one-electron
integrals and the nuclear repulsion come from the library's host code (section 4 evaluates them on
the CPU). The iterations' dense linear algebra (symmetric eigendecompositions and products of
nao x nao matrices) runs on the GPU through PyTorch's ROCm routines; the density stays on the
device. Each iteration waits for its J and K (the next density depends on them), so the work-list
check runs every iteration and a build that overflowed is redone at once. Optional Pulay DIIS on
the commutator F D S - S D F, and an optional level shift of the virtual orbitals
(F + shift (S - S D S / 2), energies from the unshifted F) for molecules whose iterations
oscillate from the core-Hamiltonian guess.
"""
from __future__ import annotations

import time

import numpy as np

from . import jk


class RHF:
    """Closed-shell SCF of a molecule (synth.Molecule fields) with nuclear charges `charges`
    (2 x occupied = sum of charges)."""

    def __init__(self, mol, charges, thresh=None, diis=8, level_shift=0.0, damping=0.0, diis_start=0,
                 precision=jk.JK_FP64, device="cuda"):
        import torch
        t = time.perf_counter()
        S, T, V, self.enuc = jk.one_electron(mol, charges)
        self.onee_s = time.perf_counter() - t
        dev = torch.device(device)
        self.S = torch.from_numpy(S).to(dev)
        self.H = torch.from_numpy(T + V).to(dev)
        s, U = torch.linalg.eigh(self.S)
        keep = s > 1e-8 * s.max()
        self.X = (U[:, keep] / torch.sqrt(s[keep])).contiguous()     # canonical orthogonalisation
        self.nocc = int(round(float(np.sum(charges)))) // 2
        t = time.perf_counter()
        self.plan = jk.Plan.from_molecule(mol, thresh=thresh, precision=precision)
        self.plan_s = time.perf_counter() - t
        self.diis = diis
        self.level_shift = level_shift     # virtual orbitals raised by this much before diagonalising
        self.damping = damping             # fraction of the previous density kept before DIIS starts
        self.diis_start = diis_start       # iteration from which DIIS extrapolates

    def density(self, F):
        import torch
        e, Cp = torch.linalg.eigh(self.X.T @ F @ self.X)
        C = self.X @ Cp[:, : self.nocc]
        D = 2.0 * C @ C.T
        return (0.5 * (D + D.T)).contiguous()

    def run(self, niter=10):
        """niter Fock builds from the core-Hamiltonian guess; returns the energy of each."""
        import torch
        D = self.density(self.H)
        J = torch.empty_like(D)
        K = torch.empty_like(D)
        energies, fs, es = [], [], []
        self.iter_ms = []
        self.overflows = 0
        torch.cuda.synchronize()
        for it in range(niter):
            t = time.perf_counter()
            self.plan.execute(D, J, K)
            try:             # the iteration needs J and K now: wait, and redo a build that overflowed
                self.plan.check()
            except jk.JKError as err:
                if err.code != jk.JK_EOVERFLOW:
                    raise
                self.overflows += 1
                self.plan.execute(D, J, K)
                self.plan.check()
            F = self.H + J - 0.5 * K
            energies.append(0.5 * torch.sum(D * (self.H + F)) + self.enuc)
            if self.diis and it >= self.diis_start:
                err = self.X.T @ (F @ D @ self.S - self.S @ D @ F) @ self.X
                fs.append(F)
                es.append(err)
                fs, es = fs[-self.diis:], es[-self.diis:]
                n = len(fs)
                B = -torch.ones((n + 1, n + 1), dtype=F.dtype, device=F.device)
                B[n, n] = 0.0
                for i in range(n):
                    for j in range(n):
                        B[i, j] = torch.sum(es[i] * es[j])
                rhs = torch.zeros(n + 1, dtype=F.dtype, device=F.device)
                rhs[n] = -1.0
                c = torch.linalg.solve(B, rhs)
                F = sum(c[i] * fs[i] for i in range(n))
            if self.level_shift:
                F = F + self.level_shift * (self.S - 0.5 * self.S @ D @ self.S)
            Dn = self.density(F)
            if self.damping and not (self.diis and it >= self.diis_start):
                Dn = (self.damping * D + (1.0 - self.damping) * Dn).contiguous()
            D = Dn
            torch.cuda.synchronize()
            self.iter_ms.append((time.perf_counter() - t) * 1e3)
        self.D = D
        return [float(e) for e in energies]

    def close(self):
        self.plan.close()
