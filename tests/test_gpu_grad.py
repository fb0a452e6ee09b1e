"""GPU: the nuclear-gradient kernels against the oracle's gradient (same screen), element by
element over atoms and directions."""
import numpy as np
import pytest

import oracle
from paper_2407_09700_amd import synth

from .gpu_util import say

pytestmark = pytest.mark.gpu


def _grad(mol, thresh=None):
    import torch
    from paper_2407_09700_amd import jk
    plan = jk.Plan.from_molecule(mol, thresh=thresh)
    D = torch.from_numpy(mol.D).cuda()
    g = plan.grad(D)
    plan.check()
    st = plan.stats()
    plan.close()
    return g.cpu().numpy(), st


def _check(mol, thresh, tag):
    g, st = _grad(mol, thresh)
    o = oracle.Oracle(mol)
    go = o.grad(tau=thresh)
    d = float(np.abs(g - go).max())
    scale = max(1.0, float(np.abs(go).max()))
    say(f"[grad {tag}] natom {mol.natom} nbf {mol.nbf} kept gpu {st['kept_quartets']} oracle {o.kept} "
        f"max|dg| {d:.2e} max|g| {np.abs(go).max():.3e}")
    assert st["kept_quartets"] == o.kept
    assert d <= 1e-10 * scale


@pytest.mark.parametrize("pure", [0, 1])
def test_grad_every_class_up_to_d(pure):
    # one contracted shell of each l <= 2 on three atoms: all 21 classes up to (dd|dd)
    coords = [[0.0, 0.0, 0.0], [1.6, 0.3, -0.5], [-0.7, 1.4, 0.8]]
    mol = synth.custom(coords, [(0, 3), (1, 2), (2, 2)], 0.25, 6.0, pure_from_l=2 if pure else 99, nocc=6, seed=60 + pure)
    _check(mol, 0.0, f"all classes pure={pure}")


def test_grad_cfg2_small_screened():
    _check(synth.make_config(2, natom=6), 1e-12, "cfg2 6 atoms")


def test_grad_translation_invariance_cfg2():
    g, _ = _grad(synth.make_config(2, natom=9), 1e-12)
    say(f"[grad sum] {g.sum(axis=0)}")
    assert np.abs(g.sum(axis=0)).max() <= 1e-9 * max(1.0, np.abs(g).max())


@pytest.mark.parametrize("pure", [0, 1])
def test_grad_every_class_up_to_f(pure):
    # one contracted shell of each l <= 3 on three atoms: all 55 classes up to (ff|ff)
    coords = [[0.0, 0.0, 0.0], [1.6, 0.3, -0.5], [-0.7, 1.4, 0.8]]
    mol = synth.custom(coords, [(0, 3), (1, 2), (2, 2), (3, 1)], 0.25, 6.0, pure_from_l=2 if pure else 99, nocc=8,
                       seed=70 + pure)
    _check(mol, 0.0, f"all classes up to f pure={pure}")


def test_grad_rejects_g_shells():
    from paper_2407_09700_amd import jk
    import torch
    mol = synth.make_config(3, natom=2)
    plan = jk.Plan.from_molecule(mol)
    with pytest.raises(jk.JKError) as e:
        plan.grad(torch.from_numpy(mol.D).cuda())
    plan.close()
    assert e.value.code == jk.JK_EUNSUPPORTED
