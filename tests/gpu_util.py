"""Helpers for the GPU parity tests: run the HIP library and the oracle on one molecule."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_jk(mol, thresh=None, D=None, repeat=1, want="jk"):
    import torch
    from paper_2407_09700_amd import jk
    plan = jk.Plan.from_molecule(mol, thresh=thresh, want=want)
    Dt = torch.from_numpy(np.ascontiguousarray(mol.D if D is None else D)).cuda()
    out = []
    for _ in range(repeat):
        J, K = plan.execute(Dt)
        plan.check()
        out.append((None if J is None else J.cpu().numpy(), None if K is None else K.cpu().numpy()))
    stats = plan.stats()
    plan.close()
    return (out if repeat > 1 else out[0]), stats


def maxabs(a, b):
    return float(np.max(np.abs(a - b))) if a.size else 0.0
