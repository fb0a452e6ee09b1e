"""GPU: the no-allocation entry point (jk_build_static) against jk_build through the C ABI,
two calls in a row (the second on a smaller molecule, over the contents the first left in the
static array), and its size limit."""
import numpy as np
import pytest

from paper_2407_09700_amd import synth

from .gpu_util import maxabs, say

pytestmark = pytest.mark.gpu


def _both(mol):
    import torch
    from paper_2407_09700_amd import jk
    D = torch.from_numpy(mol.D).cuda()
    J1, K1 = jk.build(mol, D)
    J2, K2 = jk.build(mol, D, static=True)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (J1, K1, J2, K2)]


def test_static_build_matches_jk_build_twice():
    mols = [synth.make_config(2, natom=9), synth.make_config(3, natom=2)]   # second call: smaller
    for i, mol in enumerate(mols):
        J1, K1, J2, K2 = _both(mol)
        dj, dk = maxabs(J1, J2), maxabs(K1, K2)
        say(f"[static {i}] nbf {mol.nbf}: |dJ|={dj:.2e} |dK|={dk:.2e} max|J|={np.abs(J1).max():.2e}")
        assert dj <= 1e-12 and dk <= 1e-12
        assert np.abs(J1).max() > 0 and np.abs(K1).max() > 0


def test_static_build_rejects_too_large():
    import torch
    from paper_2407_09700_amd import jk
    mol = synth.make_config(2)                 # 896 AOs: its work lists exceed the static array
    D = torch.from_numpy(mol.D).cuda()
    with pytest.raises(jk.JKError) as e:
        jk.build(mol, D, static=True)
    say(f"[static too large] {e.value}")
    assert e.value.code == jk.JK_ENOMEM and "static scratch" in str(e.value)
