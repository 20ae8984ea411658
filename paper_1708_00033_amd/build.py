"""Build the HIP library libhfx.so in-tree for gfx950.

    python -m paper_1708_00033_amd.build [-j JOBS]

Steps: generate the per-class evaluators (csrc/gen_eri.py), compile every
translation unit with hipcc in parallel, link against rocBLAS/rocSOLVER.
Every call recompiles every source.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
GEN = os.path.join(CSRC, "generated")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhfx.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
CFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-munsafe-fp-atomics",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", CSRC, "-I", INCLUDE, "-Wno-unused-command-line-argument"]


def _compile(src: str) -> tuple:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    t0 = time.time()
    cmd = [HIPCC] + CFLAGS + ["-c", src, "-o", obj]
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines() if "packed-fp32-ops" not in l and l.strip())
    return src, obj, p.returncode, out, time.time() - t0


def sources() -> list:
    gen = sorted(glob.glob(os.path.join(GEN, "eri_class_*.hip")))
    # largest classes first so the pool finishes early
    gen = sorted(gen, key=lambda s: -int(os.path.basename(s)[10:12]))
    own = [os.path.join(CSRC, f) for f in ("eri_dispatch.hip", "misc_kernels.hip", "guess.hip", "noalloc.hip", "batch_scf.hip", "hfx_api.cpp",
                                            "scf.cpp", "boys_table.cpp")]
    return gen + own


def build(jobs: int = 0, verbose: bool = True) -> str:
    subprocess.check_call([sys.executable, os.path.join(CSRC, "gen_eri.py"), GEN])
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or max(1, min(os.cpu_count() or 1, 16))
    srcs = sources()
    objs = []
    failed = []
    t0 = time.time()
    with cf.ThreadPoolExecutor(jobs) as ex:
        for src, obj, rc, out, dt in ex.map(_compile, srcs):
            if verbose:
                print(f"[build] {os.path.basename(src):24s} {dt:7.1f} s{'  FAILED' if rc else ''}", flush=True)
            if out and (rc or verbose > 1):
                print(out, flush=True)
            if rc:
                failed.append(src)
            objs.append(obj)
    if failed:
        raise RuntimeError("hipcc failed for: " + ", ".join(os.path.basename(f) for f in failed))
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs +
                          ["-L/opt/rocm/lib", "-lrocblas", "-lrocsolver", "-Wl,-rpath,/opt/rocm/lib"])
    os.replace(tmp, LIB)
    if verbose:
        print(f"[build] linked {LIB} in {time.time() - t0:.1f} s", flush=True)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", "--jobs", type=int, default=0)
    ap.add_argument("-v", "--verbose", type=int, default=1)
    a = ap.parse_args()
    build(a.jobs, a.verbose)
