"""Writes the oracle fixtures of the full-size 256-atom molecule (clustered 3s2p1d, spherical d,
3584 AOs, tau 1e-12) to tests/golden/cfg4_oracle.json. Calls only the oracle (and the input
generator); run once on the CPU:

    python tests/golden/make_oracle_fixtures.py [--threads N]

Stored: the kept quartet count of the density-weighted screen, E = tr(D (J - K/2)), tr(DJ),
tr(DK), max |J|, max |K|, and the J and K blocks of a set of shell pairs (final basis).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2407_09700_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg4_oracle.json")
# shells per atom: s6 s1 s1 p3 p1 d1 -> shell index 6*atom + k; pairs over the whole molecule
PAIRS = [(0, 0), (5, 5), (6 * 10 + 3, 6 * 2 + 0), (6 * 40 + 5, 6 * 40 + 4), (6 * 63 + 2, 6 * 17 + 1),
         (6 * 100 + 5, 6 * 5 + 5), (6 * 255 + 5, 6 * 255 + 3), (6 * 200 + 4, 6 * 199 + 1), (6 * 128 + 5, 6 * 3 + 3),
         (6 * 77 + 0, 6 * 77 + 0), (6 * 254 + 5, 6 * 1 + 5), (6 * 150 + 3, 6 * 150 + 3)]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    args = ap.parse_args()
    mol = synth.make_config(4)
    o = oracle.Oracle(mol)
    t = time.time()
    J, K = o.jk(tau=mol.thresh, nthreads=args.threads)
    dt = time.time() - t
    D = mol.D
    blocks = []
    for si, sj in PAIRS:
        sl_i = slice(int(o.off[si]), int(o.off[si + 1]))
        sl_j = slice(int(o.off[sj]), int(o.off[sj + 1]))
        blocks.append({"si": si, "sj": sj, "J": J[sl_i, sl_j].tolist(), "K": K[sl_i, sl_j].tolist()})
    out = {"workload": f"{mol.natom}-atom clustered 3s2p1d, {mol.nbf} AOs, tau {mol.thresh:g}",
           "kept_quartets": o.kept, "E": float(np.sum(D * (J - 0.5 * K))), "trDJ": float(np.sum(D * J)),
           "trDK": float(np.sum(D * K)), "max_abs_J": float(np.abs(J).max()), "max_abs_K": float(np.abs(K).max()),
           "oracle_seconds": round(dt, 1), "oracle_threads": args.threads or os.cpu_count(), "blocks": blocks}
    with open(OUT, "w") as f:
        json.dump(out, f, indent=0)
    print(f"wrote {OUT}: kept {o.kept} E {out['E']!r} in {dt:.0f}s", flush=True)


if __name__ == "__main__":
    main()
