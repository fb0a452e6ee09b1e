"""Build the HIP library libjk.so for gfx950 (in-tree, next to this file).

Usage: python -m paper_2407_09700_amd.build [-j JOBS]
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.environ.get("JK_LIB_OUT", os.path.join(HERE, "libjk.so"))
BUILD = os.environ.get("JK_BUILD_DIR", BUILD)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["jk_api.cpp", "jk_onee.cpp", "jk_aux.hip", "grad_classes.hip", "grad_classes_f.hip"] + [f"classes_{c}.hip" for c in
                                         ("44", "43", "42", "33", "41", "32", "40", "31", "22", "30", "21", "20",
                                          "11", "10", "00")]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result"]


def _stale(src: str, obj: str) -> bool:
    if not os.path.exists(obj):
        return True
    deps = [os.path.join(CSRC, src)] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    deps.append(os.path.join(HERE, "..", "include", "jk.h"))
    return max(os.path.getmtime(d) for d in deps) > os.path.getmtime(obj)


def _compile(src: str, force: bool = True) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    if not force and not _stale(src, obj):
        return obj
    cmd = [HIPCC, *FLAGS, *os.environ.get("JK_DEFINES", "").split(), "-x", "hip", "-c", os.path.join(CSRC, src),
           "-o", obj]
    if os.environ.get("JK_RESOURCE_USAGE"):
        cmd.append("-Rpass-analysis=kernel-resource-usage")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if os.environ.get("JK_RESOURCE_USAGE"):
        with open(obj + ".usage.txt", "w") as f:
            f.write(r.stderr)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = True, force: bool = True) -> str:
    """Compile every source (force=True, the default) or only stale ones, then link."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or int(os.environ.get("MAX_JOBS", "0")) or min(8, os.cpu_count() or 1)
    t0 = time.time()
    order = SOURCES[5:] + SOURCES[4:5] + SOURCES[:4]   # biggest class units first
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = dict(zip(order, ex.map(lambda s: _compile(s, force), order)))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *[objs[s] for s in SOURCES], "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f}s", flush=True)
    return LIB


if __name__ == "__main__":
    j = None
    if "-j" in sys.argv:
        j = int(sys.argv[sys.argv.index("-j") + 1])
    build(j, force="--incremental" not in sys.argv)
