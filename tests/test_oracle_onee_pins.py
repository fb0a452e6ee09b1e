"""Pins of the oracle's one-electron integrals (no GPU): closed forms for s functions,
brute-force quadrature for p and d functions, unit diagonal blocks of the normalised shells,
translation invariance; and the library's host implementation (jk_one_electron, Rys form)
against the oracle (Obara-Saika) element by element."""
import numpy as np
import pytest
from scipy.special import erf

import oracle
from paper_2407_09700_amd import synth

from .onee_bruteforce import primitive_blocks


def _two_prims(la, lb, a, b, A, B, nuclei, charges):
    """A molecule of two primitive shells (coefficient 1, Cartesian) and extra charged centres."""
    coords = np.array([A, B] + [list(c) for c in nuclei], float)
    mol = synth.Molecule(coords=coords, shell_atom=np.array([0, 1], np.int32), shell_l=np.array([la, lb], np.int32),
                         shell_nprim=np.array([1, 1], np.int32), shell_off=np.array([0, 1], np.int32),
                         shell_pure=np.zeros(2, np.int32), prim_exp=np.array([a, b]), prim_coef=np.ones(2), D=None,
                         thresh=0.0)
    Z = np.concatenate([[0.0, 0.0], charges])
    return mol, Z


def test_ss_closed_forms():
    a, b = 0.8, 1.7
    A, B, C = np.array([0.1, -0.2, 0.3]), np.array([1.0, 0.4, -0.6]), np.array([-0.5, 0.9, 0.2])
    mol, Z = _two_prims(0, 0, a, b, A, B, [C], [2.5])
    S, T, V, en = oracle.Oracle(mol).one_electron(Z)
    p = a + b
    R2 = np.sum((A - B) ** 2)
    K = np.exp(-a * b / p * R2)
    s = (np.pi / p) ** 1.5 * K
    P = (a * A + b * B) / p
    Tpc = p * np.sum((P - C) ** 2)
    F0 = 0.5 * np.sqrt(np.pi / Tpc) * erf(np.sqrt(Tpc))
    assert abs(S[0, 1] - s) <= 1e-15 * s
    assert abs(T[0, 1] - a * b / p * (3 - 2 * a * b / p * R2) * s) <= 1e-14 * s
    assert abs(V[0, 1] - (-2.5 * 2 * np.pi / p * K * F0)) <= 1e-14 * abs(V[0, 1])


@pytest.mark.parametrize("la,lb", [(1, 0), (1, 1), (2, 1), (2, 2), (3, 1)])
def test_bruteforce_primitive_blocks(la, lb):
    rng = np.random.default_rng(10 * la + lb)
    A, B = rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 3)
    nuclei = [rng.uniform(-1.5, 1.5, 3), rng.uniform(-1.5, 1.5, 3)]
    charges = [1.3, 3.0]
    a, b = rng.uniform(0.4, 1.6, 2)
    mol, Z = _two_prims(la, lb, a, b, A, B, nuclei, charges)
    S, T, V, _ = oracle.Oracle(mol).one_electron(Z)
    na = (la + 1) * (la + 2) // 2
    Sb, Tb, Vb = primitive_blocks(la, lb, a, b, A, B, nuclei, charges)
    for got, ref in ((S, Sb), (T, Tb), (V, Vb)):
        blk = got[:na, na:]
        assert np.max(np.abs(blk - ref)) <= 1e-10 * np.max(np.abs(ref)), np.max(np.abs(blk - ref))


def test_normalised_shells_have_unit_diagonal_blocks():
    # one-centre blocks of every shell of a normalised basis: identity (pure shells), unit
    # diagonal of the x^l component (Cartesian)
    mol = synth.custom([[0.0, 0.0, 0.0], [0.0, 1.5, 0.4]], [(0, 3), (1, 2), (2, 2), (3, 1), (4, 1)], 0.3, 6.0,
                       pure_from_l=2, nocc=3, seed=71)
    S, _, _, _ = oracle.Oracle(mol).one_electron(np.zeros(mol.natom))
    off = mol.ao_offsets()
    for s in range(mol.nshell):
        blk = S[off[s]:off[s + 1], off[s]:off[s + 1]]
        assert np.max(np.abs(blk - np.eye(blk.shape[0]))) <= 1e-12


def test_translation_invariance():
    mol = synth.make_config(2, natom=3)
    Z = np.full(mol.natom, 5.0)
    S, T, V, en = oracle.Oracle(mol).one_electron(Z)
    shifted = synth.Molecule(coords=mol.coords + np.array([0.7, -1.1, 2.3]), shell_atom=mol.shell_atom,
                             shell_l=mol.shell_l, shell_nprim=mol.shell_nprim, shell_off=mol.shell_off,
                             shell_pure=mol.shell_pure, prim_exp=mol.prim_exp, prim_coef=mol.prim_coef, D=mol.D,
                             thresh=mol.thresh)
    S2, T2, V2, en2 = oracle.Oracle(shifted).one_electron(Z)
    for x, y in ((S, S2), (T, T2), (V, V2)):
        assert np.max(np.abs(x - y)) <= 1e-11 * np.max(np.abs(x))
    assert abs(en - en2) <= 1e-12 * en


@pytest.mark.parametrize("pure", [0, 1])
def test_library_matches_oracle(pure):
    # jk_one_electron (host code of the library: binomial moments and a Rys rule for V) against
    # the oracle's Obara-Saika recurrences, s to g shells, contracted
    from paper_2407_09700_amd import jk
    coords = [[0.0, 0.0, 0.0], [1.7, 0.3, -0.4], [-0.6, 1.5, 1.1]]
    mol = synth.custom(coords, [(0, 3), (1, 2), (2, 2), (3, 1), (4, 2)], 0.25, 6.0, pure_from_l=2 if pure else 99,
                       nocc=9, seed=72 + pure)
    Z = np.array([3.0, 1.0, 6.0])
    So, To, Vo, eo = oracle.Oracle(mol).one_electron(Z)
    S, T, V, e = jk.one_electron(mol, Z)
    for name, x, y in (("S", S, So), ("T", T, To), ("V", V, Vo)):
        d = np.max(np.abs(x - y))
        assert d <= 1e-12 * max(1.0, np.max(np.abs(y))), (name, d)
    assert abs(e - eo) <= 1e-13 * eo
