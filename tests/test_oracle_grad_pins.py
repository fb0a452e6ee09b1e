"""Pins of the oracle's nuclear gradient (no GPU): d/dR of E = tr(D (J - K/2)) with the
density held fixed (paper section 4, the two-electron part of the gradient), checked against
finite differences of the oracle's own energy, translational invariance, and the absence of
torque for s functions."""
import numpy as np
import pytest

import oracle
from paper_2407_09700_amd import synth


def _energy(mol, coords):
    m = synth.Molecule(coords=np.array(coords), shell_atom=mol.shell_atom, shell_l=mol.shell_l,
                       shell_nprim=mol.shell_nprim, shell_off=mol.shell_off, shell_pure=mol.shell_pure,
                       prim_exp=mol.prim_exp, prim_coef=mol.prim_coef, D=mol.D, thresh=0.0)
    J, K = oracle.Oracle(m).jk(tau=0.0)
    return float(np.sum(mol.D * (J - 0.5 * K)))


def _fd_grad(mol, atoms, h=2e-3):
    """Five-point central differences (error O(h^4)) of the energy for the given atoms."""
    g = np.zeros((len(atoms), 3))
    for n, a in enumerate(atoms):
        for x in range(3):
            e = []
            for t in (-2, -1, 1, 2):
                c = np.array(mol.coords, dtype=float)
                c[a, x] += t * h
                e.append(_energy(mol, c))
            g[n, x] = (e[0] - 8 * e[1] + 8 * e[2] - e[3]) / (12 * h)
    return g


@pytest.fixture(scope="module")
def spdf_mol():
    # s, p, d and f shells (pure d and f), contracted, three atoms, a density with no symmetry
    coords = [[0.0, 0.0, 0.0], [1.6, 0.4, -0.3], [-0.5, 1.3, 0.9]]
    return synth.custom(coords, [(0, 3), (1, 2), (2, 2), (3, 1)], 0.3, 5.0, pure_from_l=2, nocc=6, seed=41)


def test_gradient_matches_finite_differences(spdf_mol):
    g = oracle.Oracle(spdf_mol).grad(tau=0.0)
    fd = _fd_grad(spdf_mol, range(spdf_mol.natom))
    scale = np.abs(g).max()
    assert scale > 1e-2
    assert np.abs(g - fd).max() <= 1e-7 * max(1.0, scale), np.abs(g - fd).max()


def test_gradient_cartesian_shells_match_finite_differences():
    coords = [[0.0, 0.0, 0.0], [0.0, 1.5, 0.7]]
    mol = synth.custom(coords, [(1, 2), (2, 1), (3, 2)], 0.4, 3.0, pure_from_l=99, nocc=4, seed=42)
    g = oracle.Oracle(mol).grad(tau=0.0)
    fd = _fd_grad(mol, [0, 1])
    assert np.abs(g - fd).max() <= 1e-7 * max(1.0, np.abs(g).max())


def test_gradient_translation_invariance(spdf_mol):
    # every centre is differentiated on its own: the forces still add up to zero
    g = oracle.Oracle(spdf_mol).grad(tau=0.0)
    assert np.abs(g.sum(axis=0)).max() <= 1e-10 * np.abs(g).max()


def test_gradient_no_torque_for_s_functions():
    # with s functions only, E does not change when the atoms rotate rigidly (D fixed), so
    # sum_A R_A x g_A = 0
    rng = np.random.default_rng(7)
    coords = rng.uniform(-1.5, 1.5, size=(4, 3))
    mol = synth.custom(coords.tolist(), [(0, 2), (0, 1)], 0.3, 4.0, nocc=3, seed=43)
    g = oracle.Oracle(mol).grad(tau=0.0)
    torque = np.cross(np.array(mol.coords), g).sum(axis=0)
    assert np.abs(torque).max() <= 1e-10 * np.abs(g).max() * np.abs(mol.coords).max()
    assert np.abs(g).max() > 1e-3


def test_gradient_rejects_g_shells():
    mol = synth.custom([[0.0, 0.0, 0.0]], [(4, 1)], 0.5, 1.0, nocc=1, seed=44)
    with pytest.raises(ValueError):
        oracle.Oracle(mol).grad(tau=0.0)
