"""Benchmark of the integral-direct J/K build on one MI355X.

A step is one jk_plan_execute on the 256-atom clustered 3s2p1d molecule (spherical d,
3584 AOs, Schwarz threshold 1e-12): density transform, block maxima, screening into
class work lists, every class kernel (Rys ERIs + contraction + digestion) and the final
symmetrise/transform. Inputs are resident in HBM; the plan (pairs + Schwarz factors) and the
first build (which sizes the work lists) come before the timed region, as an SCF reuses a plan
across iterations. Per-launch HIP events are recorded inside every timed build and read after
the timed loop (the roofline of the launch with the largest time, averaged over the steps).

Prints ONE JSON line. value = kept (screened) unique shell quartets per second. Extras: the
mixed-precision build of the same molecule (energies against the oracle's FP64 fixture), the
32-atom g-function molecule and the 64-atom molecule with their per-launch rooflines, and the
64-molecule batch.
"""
from __future__ import annotations

import argparse
import json

import numpy as np
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
    """The oracle (all host cores) on every stride-th bra shell pair of the same molecule and
    threshold: the unique quartets of those bras, screened, evaluated and digested."""
    import oracle
    o = oracle.Oracle(mol)
    ncores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    npair = mol.nshell * (mol.nshell + 1) // 2
    stride = 4096
    t = time.perf_counter()
    kept = o.jk_sample(stride, 0, nthreads=ncores)
    dt = time.perf_counter() - t
    while dt < 0.4 * target_s and stride > 1:      # sample more until the run is long enough
        stride = max(1, int(stride * max(dt, 1e-3) / target_s))
        t = time.perf_counter()
        kept = o.jk_sample(stride, 0, nthreads=ncores)
        dt = time.perf_counter() - t
    log(f"cpu baseline: stride {stride} of {npair} bra pairs, {kept} quartets in {dt:.1f}s")
    what = "every bra shell pair" if stride == 1 else f"every {stride}-th bra shell pair (index 0, {stride}, ...)"
    return {"value": kept / dt, "unit": "screened quartets/s", "cores": ncores, "kind": "oracle",
            "sample": f"unique quartets of {what} of the headline molecule ({kept} kept quartets, {dt:.1f} s, "
                      f"includes the oracle's own Schwarz/block-max setup)"}


def golden_cfg4():
    """Oracle fixture of the 256-atom molecule (tests/golden/make_oracle_fixtures.py)."""
    path = os.path.join(ROOT, "tests", "golden", "cfg4_oracle.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def _timed(fn, steps, warmup, check=None):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3 / steps
    if check is not None:
        check()
    return ms


def _energy(D, J, K):
    return float((D * (J - 0.5 * K)).sum())


def kernel_name(e):
    if e["team"] == 2:
        return "k_bra<%d,%d,%d>" % (e["la"], e["lb"], e["ld"])
    if e["team"] == 3:
        return "k_bra32<%d,%d,%d>" % (e["la"], e["lb"], e["ld"])
    return "k_cls<%d,%d,%d,%d>" % (e["la"], e["lb"], e["lc"], e["ld"])


def class_name(e):
    if e["lc"] < 0:
        return "(%d%d|**) tier %d%s" % (e["la"], e["lb"], e["ld"], " FP32" if e["team"] == 3 else "")
    return "(%d%d|%d%d)" % (e["la"], e["lb"], e["lc"], e["ld"])


def launch_table(prof):
    """Per-launch entries of a profile: time, algorithmic TFLOP/s, fraction of the FP64 peak."""
    rows = []
    for e in prof:
        if e["kind"] != 0:
            continue
        tf = e["flops"] / (e["ms"] * 1e-3) / 1e12 if e["ms"] > 0 else 0.0
        rows.append({"class": class_name(e), "kernel": kernel_name(e), "ms": round(e["ms"], 4),
                     "quartets": e["quartets"], "tflops": round(tf, 3), "frac": round(tf / PEAK_FP64_TFLOPS, 4),
                     "flops": e["flops"]})
    rows.sort(key=lambda r: -r["ms"])
    return rows


def run_config(mol, steps, warmup, precision=None, profile=True, tune=False):
    """Times `steps` builds of one molecule after `warmup` (HIP events recorded inside each build
    when profile is set; read after the timed loop, averaged over its builds)."""
    import torch
    from paper_2407_09700_amd import jk
    prec = jk.JK_FP64 if precision is None else precision
    t0 = time.perf_counter()
    plan = jk.Plan.from_molecule(mol, profile=profile, precision=prec, fp32_cutoff=1e-6, tune=tune)
    D = torch.from_numpy(mol.D).cuda()
    J = torch.empty_like(D)
    K = torch.empty_like(D)
    plan.execute(D, J, K)                          # sizes the work lists (one wait), not timed
    plan.check()
    plan_ms = (time.perf_counter() - t0) * 1e3
    for w in range(warmup):
        plan.execute(D, J, K)
    torch.cuda.synchronize()
    if profile:
        plan.profile()                             # drop the warm-up events
    t = time.perf_counter()
    for _ in range(steps):
        plan.execute(D, J, K)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3 / steps
    plan.check()
    prof = plan.profile() if profile else []
    st = plan.stats()
    E = _energy(D, J, K)
    plan.close()
    return {"ms": ms, "plan_ms": plan_ms, "stats": st, "E": E, "prof": prof}


def roofline_of(prof):
    rows = launch_table(prof)
    dom = rows[0]
    achieved = dom["flops"] / (dom["ms"] * 1e-3) / 1e12
    return {"bound": "alu", "kernel": dom["kernel"], "class": dom["class"], "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": measured_traffic(dom["kernel"]), "kernel_ms": dom["ms"]}


def breakdown_of(prof, steps_note=""):
    rows = launch_table(prof)
    class_ms = sum(r["ms"] for r in rows)
    flops = sum(r["flops"] for r in rows)
    prep = sum(e["ms"] for e in prof if e["kind"] == 1)
    fin = sum(e["ms"] for e in prof if e["kind"] == 2)
    top = [{k: v for k, v in r.items() if k != "flops"} for r in rows[:10]]
    return {"prep_ms": prep, "class_kernels_ms": class_ms, "finalize_ms": fin,
            "all_classes_tflops": flops / (class_ms * 1e-3) / 1e12 if class_ms > 0 else 0.0,
            "all_classes_frac": flops / (class_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS if class_ms > 0 else 0.0,
            "top_launches": top}


def mixed_extra(mol, fp64, steps=3):
    """FP64 build vs mixed build (FP32 below a bound of 1e-6) of the same molecule; energies
    against the oracle's FP64 build when its fixture is present."""
    from paper_2407_09700_amd import jk
    r = run_config(mol, steps, 1, precision=jk.JK_MIXED, profile=False)
    st = r["stats"]
    out = {"workload": f"{mol.natom}-atom clustered 3s2p1d, {mol.nbf} AOs, tau {mol.thresh:g}, FP32 below bound 1e-6",
           "fp64_ms": fp64["ms"], "mixed_ms": r["ms"], "speedup": fp64["ms"] / r["ms"],
           "fp32_fraction": st["kept_fp32"] / max(1, st["kept_quartets"]), "kept_quartets": st["kept_quartets"],
           "E_fp64": fp64["E"], "E_mixed": r["E"], "dE_mixed_vs_fp64_gpu": abs(r["E"] - fp64["E"])}
    g = golden_cfg4()
    if g is not None and mol.nbf == 3584:
        out["E_oracle"] = g["E"]
        out["dE_fp64_vs_oracle"] = abs(fp64["E"] - g["E"])
        out["dE_mixed_vs_oracle"] = abs(r["E"] - g["E"])
        out["kept_matches_oracle"] = st["kept_quartets"] == g["kept_quartets"]
    log(f"mixed: {r['ms']:.1f} ms vs FP64 {fp64['ms']:.1f} ms, fp32 {st['kept_fp32']} of {st['kept_quartets']}")
    return out


def batched_extra(steps=1, warmup=1):
    """64 molecules of 10-120 atoms (3s2p1d1f): one batched graph-launched build (FP64 and
    mixed) vs 64 sequential single-molecule FP64 builds."""
    import torch
    from paper_2407_09700_amd import jk, synth
    mols = synth.make_batch()
    out = {"workload": f"64 molecules, {sum(m.natom for m in mols)} atoms, "
                       f"{sum(m.nbf for m in mols)} AOs, 3s2p1d1f, tau 1e-12"}
    t = time.perf_counter()
    plans = [jk.Plan.from_molecule(m) for m in mols]
    Ds = [torch.from_numpy(m.D).cuda() for m in mols]
    Js = [torch.empty_like(d) for d in Ds]
    Ks = [torch.empty_like(d) for d in Ds]
    for p, d, j, k in zip(plans, Ds, Js, Ks):      # sizes every plan's lists (one wait each), not timed
        p.execute(d, j, k)
    log(f"batch: sequential plans in {time.perf_counter() - t:.1f}s")

    def seq():
        for p, d, j, k in zip(plans, Ds, Js, Ks):
            p.execute(d, j, k)

    def seq_check():
        for p in plans:
            p.check()
    seq_ms = _timed(seq, steps, warmup, seq_check)
    kept = sum(p.stats()["kept_quartets"] for p in plans)
    E_seq = sum(_energy(d, j, k) for d, j, k in zip(Ds, Js, Ks))
    for p in plans:
        p.close()
    out["sequential_fp64_ms"] = seq_ms
    out["kept_quartets"] = kept
    log(f"batch: sequential {seq_ms:.1f} ms, {kept} quartets")
    import tempfile
    cache = os.path.join(tempfile.gettempdir(), f"jk_tune_batch_{os.getpid()}.txt")   # FP64 tunes, mixed reuses
    for name, prec in (("fp64", jk.JK_FP64), ("mixed", jk.JK_MIXED)):
        t = time.perf_counter()
        b = jk.Batch(mols, precision=prec, graph=True, tune=True, tune_cache=cache)
        D = b.pack([m.D for m in mols])
        J = torch.empty_like(D)
        K = torch.empty_like(D)
        b.execute(D, J, K)                         # sizes, tunes, records the graph: not timed
        b.check()
        ms = _timed(lambda: b.execute(D, J, K), steps, warmup, b.check)
        E = _energy(D, J, K)
        info = b.graph_info()
        st = b.stats()
        b.close()
        log(f"batch {name}: {ms:.1f} ms (setup {time.perf_counter() - t:.1f}s) graph {info} fp32 {st['kept_fp32']}")
        out[f"batched_{name}_ms"] = ms
        out[f"batched_{name}_speedup_vs_sequential"] = seq_ms / ms
        out[f"dE_batched_{name}_vs_sequential"] = abs(E - E_seq)
        out[f"graph_replays_{name}"] = info["replays"]
    if os.path.exists(cache):
        w = open(cache).read().split()
        out["tuned"] = {w[i]: int(w[i + 1]) for i in range(0, len(w) - 1, 2)}
        os.remove(cache)
    return out


def grad_extra(steps=3, warmup=1):
    """Nuclear gradient of tr(D (J - K/2)) (jk_grad) on the 64-atom molecule, next to its J/K build."""
    import torch
    from paper_2407_09700_amd import jk, synth
    mol = synth.make_config(2)
    plan = jk.Plan.from_molecule(mol)
    D = torch.from_numpy(mol.D).cuda()
    g = plan.grad(D)
    plan.check()
    ms = _timed(lambda: plan.grad(D, out=g), steps, warmup, plan.check)
    st = plan.stats()
    plan.close()
    log(f"gradient: {ms:.1f} ms, {st['kept_quartets']} quartets")
    return {"workload": f"{mol.natom}-atom clustered 3s2p1d, {mol.nbf} AOs, tau {mol.thresh:g}", "grad_ms": ms,
            "kept_quartets": st["kept_quartets"], "quartets_per_s": st["kept_quartets"] / (ms * 1e-3),
            "max_abs_grad": float(g.abs().max())}


def scf_extra(niter=40):
    """SCF iterations on the 64-atom molecule with one plan reused: per-iteration time and the
    energies. From the core-Hamiltonian guess this synthetic molecule's plain DIIS iterations
    wander, so the first twelve iterations keep 80 % of the previous density (damping) and DIIS
    starts after them; the energy then falls monotonically."""
    from paper_2407_09700_amd import scf, synth
    mol = synth.make_config(2)
    Z = synth.nuclear_charges(mol)
    r = scf.RHF(mol, Z, diis=8, damping=0.8, diis_start=12)
    e = r.run(niter)
    it = r.iter_ms
    r.close()
    log(f"scf: {niter} iterations, {np.mean(it[1:]):.1f} ms each after the first, E {e[-1]:.8f}, "
        f"last change {abs(e[-1] - e[-2]):.2e}")
    return {"workload": f"RHF, {mol.natom}-atom clustered 3s2p1d, {mol.nbf} AOs, charges {int(Z.sum())}, damping 0.8 "
                        f"for 12 iterations then DIIS (8 vectors)",
            "iterations": niter, "iter_ms": [round(x, 2) for x in it], "mean_iter_ms_after_first": float(np.mean(it[1:])),
            "energies": e, "dE_last": abs(e[-1] - e[-2]), "plan_s": r.plan_s, "one_electron_s": r.onee_s,
            "rebuilds_after_overflow": r.overflows}


def config_extra(mol, steps, warmup, label):
    r = run_config(mol, steps, warmup)
    st = r["stats"]
    b = breakdown_of(r["prof"])
    log(f"{label}: {r['ms']:.1f} ms, {st['kept_quartets']} quartets, all launches {b['all_classes_tflops']:.2f} TF")
    return {"workload": label, "build_ms": r["ms"], "steps": steps, "kept_quartets": st["kept_quartets"],
            "quartets_per_s": st["kept_quartets"] / (r["ms"] * 1e-3), "E": r["E"], "roofline": roofline_of(r["prof"]),
            "breakdown": b}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--natom", type=int, default=None, help="smaller molecule of the same recipe (debug)")
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--tune", action="store_true", help="tune the headline plan's launches first (not timed)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the mixed-precision, g-function, 64-atom and batched measurements")
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

    from paper_2407_09700_amd import synth

    mol = synth.make_config(args.config, natom=args.natom)
    log(f"workload: config {args.config}, natom {mol.natom}, nao {mol.nbf}, nshell {mol.nshell}, tau {mol.thresh}")
    r = run_config(mol, args.steps, args.warmup, tune=args.tune)
    ms_per_step = r["ms"]
    st = r["stats"]
    kept = st["kept_quartets"]
    out = {
        "metric": METRIC, "value": kept / (ms_per_step / 1e3), "unit": "screened quartets/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded)",
        "config": {"workload": f"{mol.natom} atoms, {WORKLOAD_BASIS.get(args.config, '')}, "
                               f"{mol.nbf} AOs, Schwarz tau {mol.thresh:g}, FP64 J+K build",
                   "natom": mol.natom, "nao": mol.nbf, "nshell": mol.nshell, "tau": mol.thresh,
                   "kept_quartets": kept, "prim_quartets": st["prim_quartets"],
                   "plan_and_first_build_ms": round(r["plan_ms"], 2)},
        "roofline": roofline_of(r["prof"]),
        "breakdown": breakdown_of(r["prof"]),
    }
    log(f"headline: {ms_per_step:.1f} ms per build, {out['value']:.3e} quartets/s, dominant "
        f"{out['roofline']['kernel']} frac {out['roofline']['frac']:.3f}")
    if not args.no_extras and args.natom is None:
        if args.config == 4:
            out["mixed"] = mixed_extra(mol, r)
        out["g_functions"] = config_extra(synth.make_config(3), 1, 1,
                                          "32 atoms, uniform cube, 4s3p2d1f1g spherical, 1248 AOs, tau 1e-12, FP64")
        out["cfg_64_atoms"] = config_extra(synth.make_config(2), 10, 2,
                                           "64 atoms, 3-atom clusters, 3s2p1d (spherical d), 896 AOs, tau 1e-12, FP64")
        out["batched"] = batched_extra()
        out["scf"] = scf_extra()
        out["gradient"] = grad_extra()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(mol)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
