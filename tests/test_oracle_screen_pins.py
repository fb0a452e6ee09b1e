"""Pins of the oracle's screening tables, screening predicate and primitive contraction
(no GPU). Each one checks the oracle against an independent numpy restatement of the
definition, so that a slip in the oracle (a density block left out of the predicate, a
wrong transform of the density, a dropped contraction coefficient) fails here.

Paper section 3: the Cauchy-Schwarz factor I_ab, the pair prescreen I_ab > tau and the
density-weighted quartet test I_ab I_cd P >= tau with P the largest density element over
the six shell-pair blocks; section 2: the contracted integral as the coefficient-weighted
sum of primitive integrals.
"""
import numpy as np
import pytest

import oracle
from oracle import sph
from paper_2407_09700_amd import synth

from .bruteforce import primitive_block


def _t(l, pure):
    """Cartesian -> final-basis rows of one shell (identity for Cartesian shells)."""
    return sph.tsph(l) if (pure and l >= 2) else np.eye(synth.ncart(l))


def _dcart_blockmax(mol):
    """P[i, j] = max |(T_i^T D T_j)[a, b]| over the Cartesian components of shells i, j."""
    off = mol.ao_offsets()
    ns = mol.nshell
    Ts = [_t(int(l), int(p)) for l, p in zip(mol.shell_l, mol.shell_pure)]
    P = np.zeros((ns, ns))
    for i in range(ns):
        for j in range(ns):
            blk = Ts[i].T @ mol.D[off[i]:off[i + 1], off[j]:off[j + 1]] @ Ts[j]
            P[i, j] = np.max(np.abs(blk))
    return P


def _pairs(ns):
    return [(i, j) for i in range(ns) for j in range(i + 1)]


def _p6(P, i, j, k, l):
    return np.maximum.reduce([P[i, j], P[k, l], P[i, k], P[i, l], P[j, k], P[j, l]])


@pytest.fixture(scope="module")
def cfg2_small():
    mol = synth.make_config(2, natom=6)
    o = oracle.Oracle(mol)
    I, P = o.screen_tables()
    return mol, o, I, P


def test_density_block_maxima_match_numpy(cfg2_small):
    # pure d shells: the block maxima are of the density in the Cartesian components
    mol, o, I, P = cfg2_small
    assert mol.shell_pure.any()
    np.testing.assert_allclose(P, _dcart_blockmax(mol), rtol=1e-13, atol=1e-15)


def test_density_block_maxima_pure_g():
    # one g and one f shell per atom (pure): the transform matters for every block
    mol = synth.custom([[0.0, 0.0, 0.0], [0.0, 1.1, 1.3]], [(4, 2), (3, 1), (1, 1)], 0.3, 6.0, pure_from_l=2,
                       nocc=5, seed=77)
    _, P = oracle.Oracle(mol).screen_tables()
    np.testing.assert_allclose(P, _dcart_blockmax(mol), rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("tau", [1e-12, 1e-9, 1e-6, 1e-4])
def test_kept_count_matches_six_block_predicate(cfg2_small, tau):
    # kept iff I_ij > tau, I_kl > tau and I_ij I_kl max(P over the six blocks) >= tau,
    # unique quartets (ij) >= (kl); evaluated here with numpy on the oracle's I and P
    mol, o, I, P = cfg2_small
    pr = np.array(_pairs(mol.nshell))
    a, b = np.tril_indices(len(pr))                       # pair index a >= b
    i, j = pr[a, 0], pr[a, 1]
    k, l = pr[b, 0], pr[b, 1]
    Iij, Ikl = I[i, j], I[k, l]
    keep = (Iij > tau) & (Ikl > tau) & (Iij * Ikl * _p6(P, i, j, k, l) >= tau)
    n_np = int(np.count_nonzero(keep))
    assert o.count_kept(I, P, tau) == n_np
    o.jk(tau=tau)
    assert o.kept == n_np
    # and the predicate really uses all six blocks: with the bra and ket blocks alone,
    # fewer quartets would pass at the looser thresholds
    if tau >= 1e-6:
        two = (Iij > tau) & (Ikl > tau) & (Iij * Ikl * np.maximum(P[i, j], P[k, l]) >= tau)
        assert np.count_nonzero(two) < n_np


@pytest.mark.parametrize("want", ["j", "k"])
@pytest.mark.parametrize("tau", [1e-9, 1e-5])
def test_kept_count_matches_output_predicate(cfg2_small, want, tau):
    # J-only builds weigh the quartet by the Coulomb blocks D_ij, D_kl only; K-only builds by
    # the exchange blocks D_ik, D_il, D_jk, D_jl only (the blocks each build's updates read)
    mol, o, I, P = cfg2_small
    pr = np.array(_pairs(mol.nshell))
    a, b = np.tril_indices(len(pr))
    i, j = pr[a, 0], pr[a, 1]
    k, l = pr[b, 0], pr[b, 1]
    Iij, Ikl = I[i, j], I[k, l]
    if want == "j":
        p = np.maximum(P[i, j], P[k, l])
    else:
        p = np.maximum.reduce([P[i, k], P[i, l], P[j, k], P[j, l]])
    keep = (Iij > tau) & (Ikl > tau) & (Iij * Ikl * p >= tau)
    n_np = int(np.count_nonzero(keep))
    assert o.count_kept(I, P, tau, want=want) == n_np
    o.jk(tau=tau, want=want)
    assert o.kept == n_np
    assert n_np < o.count_kept(I, P, tau)          # fewer than the six-block screen keeps


def test_output_screen_exact_at_zero_threshold(cfg2_small):
    # with tau = 0 every quartet is kept whatever the outputs: the same J and K (up to the
    # order in which the threads' partial sums are added)
    mol, o, I, P = cfg2_small
    J3, K3 = o.jk(tau=0.0)
    n3 = o.kept
    for want in ("j", "k"):
        J1, K1 = o.jk(tau=0.0, want=want)
        assert o.kept == n3
        assert np.max(np.abs(J1 - J3)) <= 1e-13 * np.max(np.abs(J3))
        assert np.max(np.abs(K1 - K3)) <= 1e-13 * np.max(np.abs(K3))


def test_screened_minus_exact_within_dropped_bounds(cfg2_small):
    # |J(tau) - J(0)| and |K(tau) - K(0)| per element stay within the sum, over the
    # ordered quartets the predicate drops, of n_c n_d I_ab I_cd P_block (every integral
    # obeys |(ab|cd)| <= I_ab I_cd and every density element of block (c,d) <= P_cd),
    # taken to the final basis with the 1-norms of the transform rows
    mol, o, I, P = cfg2_small
    tau = 1e-6
    ns = mol.nshell
    nc = np.array([synth.ncart(int(l)) for l in mol.shell_l])
    Je, Ke = o.jk(tau=0.0)
    Js, Ks = o.jk(tau=tau)
    ii, jj, kk, ll = np.meshgrid(np.arange(ns), np.arange(ns), np.arange(ns), np.arange(ns), indexing="ij")
    Iij, Ikl = I[ii, jj], I[kk, ll]
    dropped = ~((Iij > tau) & (Ikl > tau) & (Iij * Ikl * _p6(P, ii, jj, kk, ll) >= tau))
    assert dropped.any() and not dropped.all()
    # J[a in i, b in j] sums over ordered (k, l); K[a in i, c in k] sums over ordered (j, l)
    bJ = np.einsum("ijkl,ijkl->ij", dropped, Iij * Ikl * P[kk, ll] * (nc[kk] * nc[ll]))
    bK = np.einsum("ijkl,ijkl->ik", dropped, Iij * Ikl * P[jj, ll] * (nc[jj] * nc[ll]))
    row1 = np.array([np.max(np.sum(np.abs(_t(int(l), int(p))), axis=1)) for l, p in
                     zip(mol.shell_l, mol.shell_pure)])
    off = mol.ao_offsets()
    shell_of = np.repeat(np.arange(ns), np.diff(off))
    lim_J = (row1[:, None] * row1[None, :] * bJ)[shell_of][:, shell_of]
    lim_K = (row1[:, None] * row1[None, :] * bK)[shell_of][:, shell_of]
    dJ, dK = np.abs(Js - Je), np.abs(Ks - Ke)
    assert dJ.max() > 0 and dK.max() > 0
    assert np.all(dJ <= lim_J + 1e-13) and np.all(dK <= lim_K + 1e-13)


CONTRACTED = [((1, 0, 1, 0), (3, 2, 2, 3)), ((2, 1, 1, 0), (2, 2, 3, 1)), ((3, 1, 2, 0), (2, 1, 2, 2)),
              ((3, 3, 1, 1), (1, 2, 2, 1))]


@pytest.mark.parametrize("cls,ks", CONTRACTED, ids=["".join(map(str, c)) for c, _ in CONTRACTED])
def test_contracted_block_is_coefficient_weighted_sum(cls, ks):
    # (ab|cd) = sum_{ijkl} c_i c_j c_k c_l [a_i b_j|c_k d_l] with the unnormalised
    # primitives integrated by brute-force quadrature (no recurrence, no Boys function)
    rng = np.random.default_rng(500 + sum(c * 5 ** i for i, c in enumerate(cls)))
    cen = rng.uniform(-1.0, 1.0, size=(4, 3))
    exps = [np.sort(rng.uniform(0.3, 2.5, size=k))[::-1] for k in ks]
    coefs = [rng.uniform(0.3, 1.2, size=k) * rng.choice([-1.0, 1.0], size=k) for k in ks]
    off = np.concatenate([[0], np.cumsum(ks)[:-1]]).astype(np.int32)
    mol = synth.Molecule(coords=cen, shell_atom=np.arange(4, dtype=np.int32), shell_l=np.array(cls, np.int32),
                         shell_nprim=np.array(ks, np.int32), shell_off=off, shell_pure=np.zeros(4, np.int32),
                         prim_exp=np.concatenate(exps), prim_coef=np.concatenate(coefs), D=None, thresh=0.0)
    got = oracle.Oracle(mol).eri_block(0, 1, 2, 3)
    ref = np.zeros_like(got)
    for a in range(ks[0]):
        for b in range(ks[1]):
            for c in range(ks[2]):
                for d in range(ks[3]):
                    w = coefs[0][a] * coefs[1][b] * coefs[2][c] * coefs[3][d]
                    ref += w * primitive_block(*cls, exps[0][a], exps[1][b], exps[2][c], exps[3][d], *cen, nu=80)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) <= 1e-11 * scale, np.max(np.abs(got - ref)) / scale
