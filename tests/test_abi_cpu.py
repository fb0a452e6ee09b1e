"""Host-side checks of the C-ABI library (no GPU needed): exports, argument
validation before any device call, and the library's solid-harmonic matrices."""
import ctypes

import numpy as np
import pytest

from oracle import sph
from paper_2407_09700_amd import jk, synth


def test_library_exports_every_declared_symbol():
    import re
    import os
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "jk.h")).read()
    declared = set(re.findall(r"\b(jk_[a-z_]+)\s*\(", hdr))
    assert declared == set(jk.EXPORTS)
    L = jk.lib()
    for name in declared:
        assert hasattr(L, name), name


@pytest.mark.parametrize("l", [2, 3, 4])
def test_solid_harmonics_match_oracle_fit(l):
    # library: closed form; oracle: least-squares fit of scipy's spherical harmonics
    np.testing.assert_allclose(jk.sph_matrix(l), sph.tsph(l), rtol=0, atol=5e-14)


def test_sph_matrix_rejects_bad_l():
    out = np.zeros(100)
    for l in (-1, 0, 1, 5):
        assert jk.lib().jk_sph_matrix(l, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == jk.JK_EINVAL


def _create(mol, **over):
    arrays = dict(shell_atom=mol.shell_atom.copy(), shell_l=mol.shell_l.copy(), shell_nprim=mol.shell_nprim.copy(),
                  shell_off=mol.shell_off.copy(), shell_pure=mol.shell_pure.copy(), prim_exp=mol.prim_exp.copy(),
                  prim_coef=mol.prim_coef.copy())
    coords = over.pop("coords", mol.coords.copy())
    for k, v in over.items():
        arrays[k] = v
    B = jk.BasisArrays(**arrays)
    h = ctypes.c_void_p()
    c = np.ascontiguousarray(coords, np.float64)
    rc = jk.lib().jk_plan_create(ctypes.byref(B.struct), c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 int(c.shape[0]), None, ctypes.byref(h))
    if rc == 0:
        jk.lib().jk_plan_destroy(h)
    return rc


def test_validation_errors_before_device():
    mol = synth.make_config(1)
    l = mol.shell_l.copy(); l[3] = 5
    assert _create(mol, shell_l=l) == jk.JK_EUNSUPPORTED
    n = mol.shell_nprim.copy(); n[0] = 0
    assert _create(mol, shell_nprim=n) == jk.JK_EINVAL
    a = mol.shell_atom.copy(); a[2] = 99
    assert _create(mol, shell_atom=a) == jk.JK_EINVAL
    c = mol.coords.copy(); c[1, 1] = np.nan
    assert _create(mol, coords=c) == jk.JK_EINVAL
    e = mol.prim_exp.copy(); e[4] = -1.0
    assert _create(mol, prim_exp=e) == jk.JK_EINVAL
    o = mol.shell_off.copy(); o[-1] = len(mol.prim_exp)
    assert _create(mol, shell_off=o) == jk.JK_EINVAL
    assert "shell" in jk.last_error()
    assert jk.lib().jk_plan_create(None, None, 0, None, None) == jk.JK_EINVAL
    assert jk.lib().jk_plan_execute(None, None, None, None, None) == jk.JK_EINVAL


def test_valid_input_reaches_device_check():
    import torch
    rc = _create(synth.make_config(1))
    if torch.cuda.is_available():
        assert rc == jk.JK_OK
    else:
        assert rc == jk.JK_ENODEV


def _batch_create(mols, nmol=None, opts=None):
    bases = [jk.BasisArrays.from_molecule(m) for m in mols]
    coords = [np.ascontiguousarray(m.coords, np.float64) for m in mols]
    n = len(mols) if nmol is None else nmol
    bp = (ctypes.POINTER(jk.Basis) * len(mols))(*[ctypes.pointer(b.struct) for b in bases])
    cp = (ctypes.POINTER(ctypes.c_double) * len(mols))(*[c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
                                                         for c in coords])
    na = (ctypes.c_int * len(mols))(*[c.shape[0] for c in coords])
    h = ctypes.c_void_p()
    rc = jk.lib().jk_batch_create(n, bp, cp, na, None if opts is None else ctypes.byref(opts), ctypes.byref(h))
    if rc == 0:
        jk.lib().jk_batch_destroy(h)
    return rc


def test_batch_validation_errors_before_device():
    good = synth.make_config(1, natom=2)
    bad = synth.make_config(1, natom=3)
    bad.shell_l = bad.shell_l.copy()
    bad.shell_l[0] = 7
    assert _batch_create([good, bad]) == jk.JK_EUNSUPPORTED
    assert "molecule 1" in jk.last_error()
    assert _batch_create([good], nmol=0) == jk.JK_EINVAL
    assert jk.lib().jk_batch_create(1, None, None, None, None, None) == jk.JK_EINVAL
    assert jk.lib().jk_batch_execute(None, None, None, None, None) == jk.JK_EINVAL
    assert jk.lib().jk_batch_offsets(None, None, None) == jk.JK_EINVAL
    jk.lib().jk_batch_destroy(None)          # no-op
    opts = jk.make_opts(1e-12)
    opts.flags = 64
    assert _batch_create([good], opts=opts) == jk.JK_EINVAL
    assert "flags" in jk.last_error()
    opts = jk.make_opts(-1.0)
    assert _batch_create([good], opts=opts) == jk.JK_EINVAL
