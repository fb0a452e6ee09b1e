"""GPU: mixed precision. Quartets whose density-weighted Schwarz bound is below the cutoff
are evaluated in FP32 (2D integrals, products, transfer) with FP64 roots and FP64 J/K
accumulation; everything else stays FP64."""
import numpy as np
import pytest

import oracle
from paper_2407_09700_amd import synth

from .gpu_util import maxabs, say

pytestmark = pytest.mark.gpu


def _build(mol, precision, cutoff=1e-6):
    import torch
    from paper_2407_09700_amd import jk
    plan = jk.Plan.from_molecule(mol, precision=precision, fp32_cutoff=cutoff)
    J, K = plan.execute(torch.from_numpy(mol.D).cuda())
    torch.cuda.synchronize()
    st = plan.stats()
    plan.close()
    return J.cpu().numpy(), K.cpu().numpy(), st


def _energy(D, J, K):
    return float(np.sum(D * (J - 0.5 * K)))


def test_mixed_with_zero_cutoff_is_fp64():
    from paper_2407_09700_amd import jk
    mol = synth.make_config(2, natom=9)
    J0, K0, s0 = _build(mol, jk.JK_FP64)
    J1, K1, s1 = _build(mol, jk.JK_MIXED, cutoff=0.0)
    say(f"[mixed0] kept {s1['kept_quartets']} fp32 {s1['kept_fp32']} dJ={maxabs(J0, J1):.2e} dK={maxabs(K0, K1):.2e}")
    assert s1["kept_fp32"] == 0 and s1["kept_quartets"] == s0["kept_quartets"]
    assert maxabs(J0, J1) <= 1e-13 and maxabs(K0, K1) <= 1e-13


def _fp32_count_bruteforce(mol, tau, cutoff):
    # unique shell quartets (ij) >= (kl), pairs with I > tau, tau <= I_ij I_kl P6 < cutoff,
    # with the oracle's own Schwarz factors and block maxima
    I, P = oracle.Oracle(mol).screen_tables()
    ns = mol.nshell
    pairs = [(i, j) for i in range(ns) for j in range(i + 1)]
    n = 0
    for a in range(len(pairs)):
        i, j = pairs[a]
        if I[i, j] <= tau:
            continue
        for b in range(a + 1):
            k, l = pairs[b]
            if I[k, l] <= tau:
                continue
            p = max(P[i, j], P[k, l], P[i, k], P[i, l], P[j, k], P[j, l])
            bound = I[i, j] * I[k, l] * p
            n += (tau <= bound < cutoff)
    return n


def test_mixed_routing_count_sp():
    # s and p shells only: every class has an FP32 lane body, so the FP32 count is the
    # number of kept quartets with bound below the cutoff
    from paper_2407_09700_amd import jk
    rng = np.random.default_rng(5)
    coords = rng.uniform(-7.0, 7.0, size=(7, 3))
    mol = synth.custom(coords, [(0, 3), (0, 1), (1, 2), (1, 1)], 0.2, 30.0, thresh=1e-12, nocc=6, seed=4)
    cutoff = 1e-6
    J, K, st = _build(mol, jk.JK_MIXED, cutoff)
    n32 = _fp32_count_bruteforce(mol, mol.thresh, cutoff)
    Jo, Ko = oracle.Oracle(mol).jk(tau=mol.thresh)
    say(f"[mixed sp] kept {st['kept_quartets']} fp32 {st['kept_fp32']} (brute force {n32}) "
        f"|dJ|={maxabs(J, Jo):.2e} |dK|={maxabs(K, Ko):.2e}")
    assert st["kept_fp32"] == n32 and n32 > 0
    assert maxabs(J, Jo) <= 1e-9 and maxabs(K, Ko) <= 1e-9


def test_mixed_error_cfg2_small():
    from paper_2407_09700_amd import jk
    mol = synth.make_config(2, natom=6)
    J, K, st = _build(mol, jk.JK_MIXED, 1e-6)
    Jo, Ko = oracle.Oracle(mol).jk(tau=mol.thresh)
    dE = abs(_energy(mol.D, J, K) - _energy(mol.D, Jo, Ko))
    say(f"[mixed cfg2] kept {st['kept_quartets']} fp32 {st['kept_fp32']} "
        f"|dJ|={maxabs(J, Jo):.2e} |dK|={maxabs(K, Ko):.2e} |dE|={dE:.2e}")
    assert st["kept_fp32"] > 0
    # each FP32 quartet has |(ab|cd)| <= I_ab I_cd and bound < cutoff: its error is a few
    # FP32 ulps of quantities below the cutoff, far inside these limits
    assert maxabs(J, Jo) <= 1e-9 and maxabs(K, Ko) <= 1e-9 and dE <= 1e-8


def test_mixed_large_cutoff_stays_close():
    # route almost every lane-body quartet to FP32 (cutoff far above the bounds): the result
    # is then limited by FP32 itself (relative ~1e-6 of the largest integrals)
    from paper_2407_09700_amd import jk
    mol = synth.make_config(3, natom=2)
    J, K, st = _build(mol, jk.JK_MIXED, cutoff=1e30)
    Jo, Ko = oracle.Oracle(mol).jk(tau=mol.thresh)
    rel = max(maxabs(J, Jo) / np.max(np.abs(Jo)), maxabs(K, Ko) / np.max(np.abs(Ko)))
    say(f"[mixed all] fp32 {st['kept_fp32']} of {st['kept_quartets']} rel err {rel:.2e}")
    assert 0 < st["kept_fp32"] < st["kept_quartets"]     # the workgroup-body classes stay FP64
    assert rel <= 1e-4
