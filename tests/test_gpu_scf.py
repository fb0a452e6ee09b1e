"""GPU: SCF iterations around the J/K build against the reference iterations built from the
oracle's integrals (numpy linear algebra), energy by energy."""
import numpy as np
import pytest

from paper_2407_09700_amd import synth

from .gpu_util import say
from .scf_reference import rhf

pytestmark = pytest.mark.gpu


def test_scf_roothaan_matches_reference():
    from paper_2407_09700_amd import scf
    mol = synth.make_config(2, natom=3)
    Z = synth.nuclear_charges(mol)
    ref = rhf(mol, Z, niter=12, diis=0)
    r = scf.RHF(mol, Z, diis=0)
    e = np.array(r.run(12))
    r.close()
    say(f"[scf roothaan] energies {e[-3:]} reference {ref[-3:]} max diff {np.abs(e - ref).max():.2e}")
    assert np.abs(e - ref).max() <= 1e-8
    assert abs(e[-1] - e[-2]) <= 1e-8          # converged


def test_scf_diis_matches_reference():
    from paper_2407_09700_amd import scf
    mol = synth.make_config(2, natom=6)
    Z = synth.nuclear_charges(mol)
    ref = rhf(mol, Z, niter=15, diis=8)
    r = scf.RHF(mol, Z, diis=8)
    e = np.array(r.run(15))
    r.close()
    say(f"[scf diis] energies {e[-3:]} reference {ref[-3:]} max diff {np.abs(e - ref).max():.2e}")
    assert np.abs(e - ref).max() <= 1e-6


def test_scf_level_shift_matches_reference():
    from paper_2407_09700_amd import scf
    mol = synth.make_config(2, natom=6)
    Z = synth.nuclear_charges(mol)
    ref = rhf(mol, Z, niter=12, diis=8, level_shift=0.5)
    r = scf.RHF(mol, Z, diis=8, level_shift=0.5)
    e = np.array(r.run(12))
    r.close()
    say(f"[scf shift] energies {e[-3:]} reference {ref[-3:]} max diff {np.abs(e - ref).max():.2e}")
    assert np.abs(e - ref).max() <= 1e-6
