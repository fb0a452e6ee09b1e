"""Benchmark of the integral-direct J/K build on one MI355X.

A step is one jk_plan_execute on the 64-atom clustered 3s2p1d molecule (spherical d,
896 AOs, Schwarz threshold 1e-12): density transform, block maxima, screening into
class work lists, every class kernel (Rys ERIs + contraction + digestion) and the final
symmetrise/transform. Inputs are resident in HBM; the plan (pairs + Schwarz factors) is
built once before the timed region, as an SCF would reuse it across iterations.

Prints ONE JSON line. value = kept (screened) unique shell quartets per second.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 vector: 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
METRIC = "J+K build ms and screened quartets/s; FP32-mixed & batched vs FP64 at stated dE"
WORKLOAD_BASIS = {1: "uniform cube, 3s1p Cartesian", 2: "3-atom clusters, 3s2p1d (spherical d)",
                  3: "uniform cube, 4s3p2d1f1g spherical", 4: "3-atom clusters, 3s2p1d (spherical d)"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# HBM traffic of the dominant kernel from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE),
# scaled by the same counters read for a plain copy of known size (bench.py --copy-probe).
# Valid only for the kernel sources it was taken from: SOURCE_HASH is the hash of csrc/ then.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.txt")


def source_hash():
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2407_09700_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".h", ".hip", ".cpp")):
            with open(os.path.join(d, f), "rb") as fh:
                h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """Bytes per launch of `kernel` from profiles/traffic.txt (lines 'key value'), or None
    when the file is absent, names another kernel or was taken from other sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        parts = line.split()
        if len(parts) == 2 and not line.startswith("#"):
            kv[parts[0]] = parts[1]
    if kv.get("kernel") != kernel or kv.get("source_hash") != source_hash():
        return None
    try:
        return float(kv["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_probe(nbytes):
    """A plain device copy of nbytes (calibration of the FETCH_SIZE / WRITE_SIZE counters)."""
    import torch
    n = nbytes // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 8, "launches": 5}), flush=True)


def cpu_baseline(mol, target_s=12.0):
    import oracle
    o = oracle.Oracle(mol)
    ncores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    t = time.perf_counter()
    n = o.jk_sample(256, 0, nthreads=ncores)
    probe = time.perf_counter() - t
    rate = max(n, 1) / max(probe, 1e-3)
    npair = mol.nshell * (mol.nshell + 1) // 2
    total_est = rate and (n * 256)                      # rough kept count of the full build
    stride = max(1, int(round(256 * probe / target_s)))
    t = time.perf_counter()
    kept = o.jk_sample(stride, 1, nthreads=ncores)
    dt = time.perf_counter() - t
    if dt < 0.4 * target_s and stride > 1:          # the small probe overstated the cost: sample more
        stride = max(1, int(stride * dt / target_s))
        t = time.perf_counter()
        kept = o.jk_sample(stride, 1, nthreads=ncores)
        dt = time.perf_counter() - t
    log(f"cpu baseline: stride {stride} of {npair} bra pairs, {kept} quartets in {dt:.1f}s (est. full {total_est})")
    return {"value": kept / dt, "unit": "screened quartets/s", "cores": ncores, "kind": "oracle",
            "sample": f"unique quartets of every {stride}-th bra shell pair ({kept} kept quartets, {dt:.1f} s, "
                      f"includes the oracle's own Schwarz/block-max setup)"}


def _timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) * 1e3 / steps


def _energy(D, J, K):
    return float((D * (J - 0.5 * K)).sum())


def mixed_extra(steps=2, warmup=1):
    """256-atom clustered 3s2p1d molecule: FP64 build vs mixed build (FP32 below 1e-6)."""
    import torch
    from paper_2407_09700_amd import jk, synth
    mol = synth.make_config(4)
    D = torch.from_numpy(mol.D).cuda()
    out = {"workload": f"cfg4: {mol.natom}-atom clustered 3s2p1d, {mol.nbf} AOs, tau {mol.thresh:g}, "
                       f"FP32 below bound 1e-6"}
    res = {}
    for name, prec in (("fp64", jk.JK_FP64), ("mixed", jk.JK_MIXED)):
        plan = jk.Plan.from_molecule(mol, precision=prec, fp32_cutoff=1e-6)
        J = torch.empty_like(D)
        K = torch.empty_like(D)
        ms = _timed(lambda: plan.execute(D, J, K), steps, warmup)
        st = plan.stats()
        res[name] = (ms, _energy(D, J, K), st)
        plan.close()
        log(f"cfg4 {name}: {ms:.1f} ms kept {st['kept_quartets']} fp32 {st['kept_fp32']}")
    out.update({"fp64_ms": res["fp64"][0], "mixed_ms": res["mixed"][0],
                "speedup": res["fp64"][0] / res["mixed"][0],
                "fp32_fraction": res["mixed"][2]["kept_fp32"] / max(1, res["mixed"][2]["kept_quartets"]),
                "kept_quartets": res["fp64"][2]["kept_quartets"],
                "E_fp64": res["fp64"][1], "dE_mixed_vs_fp64": abs(res["mixed"][1] - res["fp64"][1])})
    return out


def batched_extra(steps=1, warmup=1):
    """64 molecules of 10-120 atoms (3s2p1d1f): one batched graph-replayed build (FP64 and
    mixed) vs 64 sequential single-molecule FP64 builds."""
    import torch
    from paper_2407_09700_amd import jk, synth
    mols = synth.make_batch()
    out = {"workload": f"cfg5: {len(mols)} molecules, {sum(m.natom for m in mols)} atoms, "
                       f"{sum(m.nbf for m in mols)} AOs, 3s2p1d1f, tau 1e-12"}
    t = time.perf_counter()
    plans = [jk.Plan.from_molecule(m) for m in mols]
    Ds = [torch.from_numpy(m.D).cuda() for m in mols]
    Js = [torch.empty_like(d) for d in Ds]
    Ks = [torch.empty_like(d) for d in Ds]
    log(f"cfg5 sequential plans in {time.perf_counter() - t:.1f}s")

    def seq():
        for p, d, j, k in zip(plans, Ds, Js, Ks):
            p.execute(d, j, k)
    seq_ms = _timed(seq, steps, warmup)
    kept = sum(p.stats()["kept_quartets"] for p in plans)
    E_seq = sum(_energy(d, j, k) for d, j, k in zip(Ds, Js, Ks))
    for p in plans:
        p.close()
    out["sequential_fp64_ms"] = seq_ms
    out["kept_quartets"] = kept
    log(f"cfg5 sequential: {seq_ms:.1f} ms, {kept} quartets")
    import tempfile
    cache = os.path.join(tempfile.gettempdir(), f"jk_tune_cfg5_{os.getpid()}.txt")   # FP64 tunes, mixed reuses
    for name, prec in (("fp64", jk.JK_FP64), ("mixed", jk.JK_MIXED)):
        t = time.perf_counter()
        b = jk.Batch(mols, precision=prec, graph=True, tune=True, tune_cache=cache)
        D = b.pack([m.D for m in mols])
        J = torch.empty_like(D)
        K = torch.empty_like(D)
        ms = _timed(lambda: b.execute(D, J, K), steps, warmup + 1)   # +1: the first execute records the graph
        E = _energy(D, J, K)
        info = b.graph_info()
        st = b.stats()
        b.close()
        log(f"cfg5 batched {name}: {ms:.1f} ms (setup {time.perf_counter() - t:.1f}s) graph {info} "
            f"fp32 {st['kept_fp32']}")
        out[f"batched_{name}_ms"] = ms
        out[f"batched_{name}_speedup_vs_sequential"] = seq_ms / ms
        out[f"dE_batched_{name}_vs_sequential"] = abs(E - E_seq)
        out[f"graph_replays_{name}"] = info["replays"]
    if os.path.exists(cache):
        w = open(cache).read().split()
        out["tuned_grids"] = {w[i]: int(w[i + 1]) for i in range(0, len(w) - 1, 2)}
    if os.path.exists(cache):
        os.remove(cache)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--natom", type=int, default=None, help="smaller molecule of the same recipe (debug)")
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--no-extras", action="store_true", help="skip the mixed-precision and batched measurements")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter calibration) and exit")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1:
        print(f"bench.py: the J/K path runs on one GPU only (--gpus {args.gpus} requested); it "
              f"would shard by bra-pair tiles with one all-reduce of J and K, which is not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2407_09700_amd import jk, synth

    mol = synth.make_config(args.config, natom=args.natom)
    log(f"workload: config {args.config}, natom {mol.natom}, nao {mol.nbf}, nshell {mol.nshell}, tau {mol.thresh}")
    t0 = time.perf_counter()
    plan = jk.Plan.from_molecule(mol, profile=True)
    plan_ms = (time.perf_counter() - t0) * 1e3
    D = torch.from_numpy(mol.D).cuda()
    J = torch.empty_like(D)
    K = torch.empty_like(D)
    stream = torch.cuda.current_stream()

    for w in range(args.warmup):
        plan.execute(D, J, K)
        torch.cuda.synchronize()
        log(f"warmup {w} done")

    per_class = {}
    prep_ms = fin_ms = 0.0
    t = time.perf_counter()
    for k in range(args.steps):
        plan.execute(D, J, K)
        if args.steps <= 3:
            log(f"step {k} enqueued")
        for e in plan.profile():          # HIP events recorded on this stream inside the step
            if e["kind"] == 1:
                prep_ms += e["ms"]
            elif e["kind"] == 2:
                fin_ms += e["ms"]
            else:
                key = (e["la"], e["lb"], e["lc"], e["ld"], e["team"])
                acc = per_class.setdefault(key, dict(ms=0.0, flops=0.0, quartets=0, prim=0, team=e["team"]))
                acc["ms"] += e["ms"]
                acc["flops"] += e["flops"]
                acc["quartets"] += e["quartets"]
                acc["prim"] += e["prim_quartets"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    ms_per_step = elapsed * 1e3 / args.steps
    st = plan.stats()
    kept = st["kept_quartets"]
    value = kept / (ms_per_step / 1e3)

    # dominant kernel: the class launch with the largest total time
    dom_key, dom = max(per_class.items(), key=lambda kv: kv[1]["ms"])
    dom_ms = dom["ms"] / args.steps
    achieved = dom["flops"] / args.steps / (dom_ms * 1e-3) / 1e12
    tot_flops = sum(v["flops"] for v in per_class.values()) / args.steps
    class_ms = sum(v["ms"] for v in per_class.values()) / args.steps
    top = sorted(per_class.items(), key=lambda kv: -kv[1]["ms"])[:8]
    def cname(k):
        if k[2] < 0:
            return "(%d%d|**) tier %d%s" % (k[0], k[1], k[3], " FP32" if k[4] == 3 else "")
        return "(%d%d|%d%d)" % k[:4]

    def kname(k, v):
        if v["team"] == 2:
            return "k_bra<%d,%d,%d>" % (k[0], k[1], k[3])
        if v["team"] == 3:
            return "k_bra32<%d,%d,%d>" % (k[0], k[1], k[3])
        return "k_cls<%d,%d,%d,%d>" % k[:4] + (" team" if v["team"] else " lane")

    classes = [{"class": cname(k), "kernel": kname(k, v),
                "ms": round(v["ms"] / args.steps, 4), "quartets": v["quartets"] // args.steps,
                "tflops": round(v["flops"] / v["ms"] * 1e-9, 3) if v["ms"] > 0 else 0.0} for k, v in top]

    out = {
        "metric": METRIC, "value": value, "unit": "screened quartets/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded)",
        "config": {"workload": f"cfg{args.config}: {mol.natom} atoms, {WORKLOAD_BASIS.get(args.config, '')}, "
                               f"{mol.nbf} AOs, Schwarz tau {mol.thresh:g}, FP64",
                   "natom": mol.natom, "nao": mol.nbf, "nshell": mol.nshell, "tau": mol.thresh,
                   "kept_quartets": kept, "prim_quartets": st["prim_quartets"], "plan_ms": round(plan_ms, 2)},
        "roofline": {"bound": "alu", "kernel": kname(dom_key, dom),
                     "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": measured_traffic(kname(dom_key, dom)),
                     "kernel_ms": dom_ms},
        "breakdown": {"prep_ms": prep_ms / args.steps, "class_kernels_ms": class_ms,
                      "finalize_ms": fin_ms / args.steps, "all_classes_tflops": tot_flops / (class_ms * 1e-3) / 1e12,
                      "top_classes": classes},
    }
    plan.close()
    if not args.no_extras and args.natom is None:
        out["mixed"] = mixed_extra()
        out["batched"] = batched_extra()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(mol)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
