"""Pins of the CPU oracle against facts fixed by the mathematics (no GPU).

Each test would fail for a plausible slip in the oracle: a dropped VRR/HRR term, a wrong
index or sign, a transposed operand, a wrong prefactor or a wrong J/K index pattern.
"""
import math

import numpy as np
import pytest
from scipy.special import erf, eval_legendre, gamma, gammainc

import oracle
from oracle import sph
from paper_2407_09700_amd import synth

from .bruteforce import primitive_block


# ----------------------------------------------------------------------- Boys function

@pytest.mark.parametrize("T", [1e-3, 0.1, 0.9, 3.0, 7.5, 17.0, 29.0, 44.99, 45.01, 60.0, 150.0, 800.0])
def test_boys_matches_incomplete_gamma(T):
    F = oracle.boys(16, T)
    ref = np.array([gamma(m + 0.5) * gammainc(m + 0.5, T) / (2.0 * T ** (m + 0.5)) for m in range(17)])
    np.testing.assert_allclose(F, ref, rtol=3e-14, atol=0)


def test_boys_limits():
    np.testing.assert_array_equal(oracle.boys(16, 0.0), 1.0 / (2 * np.arange(17) + 1))
    F = oracle.boys(0, 2.7)
    assert abs(F[0] - 0.5 * math.sqrt(math.pi / 2.7) * math.erf(math.sqrt(2.7))) < 1e-15


# ----------------------------------------------------------------------- primitive ERIs

def _prim_mol(ls, exps, centres, pure=0):
    """Molecule with one primitive shell per centre, coefficient 1 (unnormalised)."""
    n = len(ls)
    return synth.Molecule(coords=np.array(centres, float), shell_atom=np.arange(n, dtype=np.int32),
                          shell_l=np.array(ls, np.int32), shell_nprim=np.ones(n, np.int32),
                          shell_off=np.arange(n, dtype=np.int32), shell_pure=np.full(n, pure, np.int32),
                          prim_exp=np.array(exps, float), prim_coef=np.ones(n), D=None, thresh=0.0)


def test_ssss_closed_form():
    rng = np.random.default_rng(11)
    for _ in range(20):
        ex = rng.uniform(0.05, 20.0, size=4)
        cen = rng.uniform(-2, 2, size=(4, 3))
        o = oracle.Oracle(_prim_mol([0, 0, 0, 0], ex, cen))
        a, b, c, d = ex
        A, B, C, D = cen
        p, q = a + b, c + d
        P = (a * A + b * B) / p
        Q = (c * C + d * D) / q
        T = p * q / (p + q) * np.sum((P - Q) ** 2)
        F0 = 1.0 if T < 1e-14 else 0.5 * math.sqrt(math.pi / T) * erf(math.sqrt(T))
        ref = 2 * math.pi ** 2.5 / (p * q * math.sqrt(p + q)) * math.exp(-a * b / p * np.sum((A - B) ** 2)) \
            * math.exp(-c * d / q * np.sum((C - D) ** 2)) * F0
        got = o.eri_block(0, 1, 2, 3)[0, 0, 0, 0]
        assert abs(got - ref) <= 1e-14 * abs(ref)


CLASSES = [(1, 0, 0, 0), (1, 1, 0, 0), (1, 0, 1, 0), (1, 1, 1, 1), (2, 0, 0, 0), (2, 1, 1, 0), (2, 2, 1, 1),
           (0, 2, 1, 2), (3, 0, 1, 0), (3, 2, 0, 1), (4, 0, 0, 0), (0, 4, 1, 1), (3, 3, 2, 1), (4, 4, 2, 2),
           (4, 3, 4, 3), (4, 4, 4, 4)]


@pytest.mark.parametrize("cls", CLASSES, ids=["".join(map(str, c)) for c in CLASSES])
def test_primitive_block_vs_bruteforce(cls):
    rng = np.random.default_rng(100 + sum(c * 7 ** i for i, c in enumerate(cls)))
    ex = rng.uniform(0.3, 2.5, size=4)
    cen = rng.uniform(-1.0, 1.0, size=(4, 3))
    o = oracle.Oracle(_prim_mol(list(cls), ex, cen))
    got = o.eri_block(0, 1, 2, 3)
    ref = primitive_block(*cls, *ex, *cen)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) <= 1e-11 * scale, np.max(np.abs(got - ref)) / scale


def test_coincident_centres_and_zero_distance():
    # all four on one centre (T = 0 everywhere) against brute force
    ex = [0.7, 1.3, 0.4, 2.2]
    cen = [[0.1, -0.2, 0.3]] * 4
    o = oracle.Oracle(_prim_mol([2, 1, 2, 1], ex, cen))
    ref = primitive_block(2, 1, 2, 1, *ex, *np.array(cen))
    assert np.max(np.abs(o.eri_block(0, 1, 2, 3) - ref)) <= 1e-11 * np.max(np.abs(ref))
    # odd total angular momentum on a single centre vanishes by parity
    o = oracle.Oracle(_prim_mol([2, 1, 2, 0], ex, cen))
    assert np.max(np.abs(o.eri_block(0, 1, 2, 3))) == 0.0


# ----------------------------------------------------------------------- symmetry / Schwarz / J,K

@pytest.fixture(scope="module")
def cfg1():
    mol = synth.make_config(1)
    o = oracle.Oracle(mol)
    return mol, o, o.eri_tensor()


def test_eightfold_symmetry(cfg1):
    _, _, E = cfg1
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0)]:
        assert np.max(np.abs(E - E.transpose(perm))) <= 1e-14 * np.max(np.abs(E))


def test_schwarz_inequality(cfg1):
    _, o, E = cfg1
    n = E.shape[0]
    diag = np.einsum("ijij->ij", E)
    assert np.all(diag >= -1e-15)
    bound = np.sqrt(np.abs(diag))
    assert np.all(np.abs(E) <= bound[:, :, None, None] * bound[None, None, :, :] * (1 + 1e-12) + 1e-16)
    I = o.schwarz()
    off = o.off
    for i in range(o.ns):
        for j in range(o.ns):
            assert abs(I[i, j] - np.sqrt(diag[off[i]:off[i + 1], off[j]:off[j + 1]].max())) < 1e-14


def test_jk_loops_match_einsum(cfg1):
    mol, o, E = cfg1
    J, K = o.jk(tau=0.0)
    Jr = np.einsum("ijkl,kl->ij", E, mol.D)
    Kr = np.einsum("ikjl,kl->ij", E, mol.D)
    assert np.max(np.abs(J - Jr)) < 1e-13 * np.max(np.abs(Jr)) * 10
    assert np.max(np.abs(K - Kr)) < 1e-13 * np.max(np.abs(Kr)) * 10
    assert o.kept == 300 * 301 // 2


def test_jk_block_matches_full(cfg1):
    mol, o, _ = cfg1
    J, K = o.jk(tau=0.0)
    for si, sj in [(0, 0), (3, 1), (7, 22), (23, 23)]:
        Jb, Kb = o.jk_block(si, sj, tau=0.0)
        sl_i = slice(o.off[si], o.off[si + 1])
        sl_j = slice(o.off[sj], o.off[sj + 1])
        assert np.max(np.abs(Jb - J[sl_i, sl_j])) < 1e-12
        assert np.max(np.abs(Kb - K[sl_i, sl_j])) < 1e-12


def test_energies_positive_and_ordered(cfg1):
    mol, o, _ = cfg1
    J, K = o.jk(tau=0.0)
    ej, ek = np.sum(mol.D * J), np.sum(mol.D * K)
    assert ej >= ek >= 0.0
    assert np.max(np.abs(J - J.T)) < 1e-13 and np.max(np.abs(K - K.T)) < 1e-13


def test_linearity_and_zero_density(cfg1):
    mol, o, _ = cfg1
    rng = np.random.default_rng(5)
    D2 = rng.normal(size=mol.D.shape)
    D2 = D2 + D2.T
    J1, K1 = o.jk(D=mol.D, tau=0.0)
    J2, K2 = o.jk(D=D2, tau=0.0)
    J3, K3 = o.jk(D=mol.D + 0.5 * D2, tau=0.0)
    assert np.max(np.abs(J3 - (J1 + 0.5 * J2))) < 1e-12
    assert np.max(np.abs(K3 - (K1 + 0.5 * K2))) < 1e-12
    J0, K0 = o.jk(D=np.zeros_like(mol.D), tau=0.0)
    assert not J0.any() and not K0.any()


# ----------------------------------------------------------------------- spherical functions

@pytest.mark.parametrize("l", [2, 3, 4])
def test_sph_rows_are_harmonic(l):
    T = sph.tsph(l)
    comps = sph.cart_components(l)
    # Laplacian of sum_c T[m,c] x^a y^b z^c must vanish identically
    lap = {}
    for m in range(2 * l + 1):
        lap.clear()
        for coef, (a, b, c) in zip(T[m], comps):
            for k, (e, idx) in enumerate([(a, 0), (b, 1), (c, 2)]):
                if e >= 2:
                    key = [a, b, c]
                    key[idx] -= 2
                    lap[tuple(key)] = lap.get(tuple(key), 0.0) + coef * e * (e - 1)
        assert all(abs(v) < 1e-12 for v in lap.values())


@pytest.mark.parametrize("l", [2, 3, 4])
def test_sph_m0_row_is_legendre(l):
    T = sph.tsph(l)
    rng = np.random.default_rng(3)
    v = rng.normal(size=(50, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    comps = sph.cart_components(l)
    poly = sum(T[l, k] * v[:, 0] ** a * v[:, 1] ** b * v[:, 2] ** c for k, (a, b, c) in enumerate(comps))
    leg = eval_legendre(l, v[:, 2])
    assert np.max(np.abs(np.abs(poly) - np.abs(leg))) < 1e-13


def _one_centre_overlap(l, exps, coefs):
    comps = sph.cart_components(l)

    def mom(n, s):
        if n % 2:
            return 0.0
        df = 1.0
        k = n - 1
        while k > 1:
            df *= k
            k -= 2
        return df / (2 * s) ** (n // 2) * math.sqrt(math.pi / s)

    S = np.zeros((len(comps), len(comps)))
    for i, ci in enumerate(comps):
        for j, cj in enumerate(comps):
            tot = 0.0
            for ea, ca in zip(exps, coefs):
                for eb, cb in zip(exps, coefs):
                    s = ea + eb
                    tot += ca * cb * mom(ci[0] + cj[0], s) * mom(ci[1] + cj[1], s) * mom(ci[2] + cj[2], s)
            S[i, j] = tot
    return S


@pytest.mark.parametrize("cfg", [2, 3])
def test_spherical_functions_orthonormal(cfg):
    mol = synth.make_config(cfg, natom=1)
    for s in range(mol.nshell):
        l = int(mol.shell_l[s])
        e = mol.prim_exp[mol.shell_off[s]:mol.shell_off[s] + mol.shell_nprim[s]]
        c = mol.prim_coef[mol.shell_off[s]:mol.shell_off[s] + mol.shell_nprim[s]]
        S = _one_centre_overlap(l, e, c)
        assert abs(S[0, 0] - 1.0) < 1e-13                      # x^l component unit norm
        if l >= 2:
            T = sph.tsph(l)
            assert np.max(np.abs(T @ S @ T.T - np.eye(2 * l + 1))) < 1e-12


# ----------------------------------------------------------------------- invariances

def _rotation(seed):
    rng = np.random.default_rng(seed)
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _shell_rotation(l, pure, R):
    """U with phi(R^-1 v) = phi(v) U for the shell's angular functions, by least squares."""
    rng = np.random.default_rng(9)
    v = rng.normal(size=(200, 3))
    comps = sph.cart_components(l)

    def phi(pts):
        m = np.stack([pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c for a, b, c in comps], axis=1)
        return m @ sph.tsph(l).T if (pure and l >= 2) else m

    U, *_ = np.linalg.lstsq(phi(v), phi(v @ R), rcond=None)     # rows of v @ R are R^T v = R^-1 v
    return U


def _rotate(mol, R, shift):
    U = np.zeros((mol.nbf, mol.nbf))
    off = mol.ao_offsets()
    for s in range(mol.nshell):
        U[off[s]:off[s + 1], off[s]:off[s + 1]] = _shell_rotation(int(mol.shell_l[s]), int(mol.shell_pure[s]), R)
    rot = synth.Molecule(coords=mol.coords @ R.T + shift, shell_atom=mol.shell_atom, shell_l=mol.shell_l,
                         shell_nprim=mol.shell_nprim, shell_off=mol.shell_off, shell_pure=mol.shell_pure,
                         prim_exp=mol.prim_exp, prim_coef=mol.prim_coef, D=U @ mol.D @ U.T, thresh=mol.thresh)
    return rot


@pytest.mark.parametrize("pure", [0, 1])
def test_rotation_invariance_high_l(pure):
    coords = [[0.0, 0.0, 0.0], [1.9, 0.4, -0.3], [-0.5, 1.7, 0.9]]
    mol = synth.custom(coords, [(0, 2), (1, 1), (2, 2), (3, 1), (4, 1)], 0.3, 4.0, pure_from_l=2 if pure else 99,
                       nocc=6, seed=4)
    J, K = oracle.Oracle(mol).jk(tau=0.0)
    rot = _rotate(mol, _rotation(17), np.array([0.3, -1.1, 2.0]))
    Jr, Kr = oracle.Oracle(rot).jk(tau=0.0)
    ej, ek = np.sum(mol.D * J), np.sum(mol.D * K)
    assert abs(np.sum(rot.D * Jr) - ej) < 1e-11 * abs(ej)
    assert abs(np.sum(rot.D * Kr) - ek) < 1e-11 * abs(ek)


def test_translation_invariance():
    mol = synth.make_config(3, natom=3)
    J, K = oracle.Oracle(mol).jk(tau=0.0)
    moved = _rotate(mol, np.eye(3), np.array([5.0, -3.0, 1.5]))
    Jt, Kt = oracle.Oracle(moved).jk(tau=0.0)
    assert np.max(np.abs(J - Jt)) < 1e-11 and np.max(np.abs(K - Kt)) < 1e-11


def test_screening_tau_zero_is_exact_and_bounded():
    mol = synth.make_config(2, natom=6)
    o = oracle.Oracle(mol)
    Je, Ke = o.jk(tau=0.0)
    Js, Ks = o.jk(tau=1e-8)
    assert o.kept < o.ns * (o.ns + 1) // 2 * (o.ns * (o.ns + 1) // 2 + 1) // 2
    # each dropped quartet changes an element by at most a few bounds; 1e-8 * count is loose
    assert np.max(np.abs(Je - Js)) < 1e-5 and np.max(np.abs(Ke - Ks)) < 1e-5
