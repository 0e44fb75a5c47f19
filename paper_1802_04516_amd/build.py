"""Build libsdg.so (HIP kernels for gfx950 + host setup + C ABI) in-tree.

    python -m paper_1802_04516_amd.build [--jobs N]

Every .hip unit is compiled for gfx950 only.  Packed FP32 instructions are
disabled for all device code.  Object files go to csrc/_build/ (ignored by
git); the shared library is written next to this file.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(CSRC, "_build")
LIB = os.path.join(HERE, "libsdg.so")
ARCH = "gfx950"

COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
          "-Wno-unused-result"]
DEVICE = ["-x", "hip", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-munsafe-fp-atomics"]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm is required to build the HIP library)")


def sources():
    hip = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    cpp = sorted(f for f in os.listdir(CSRC) if f.endswith(".cpp"))
    return hip, cpp


def _compile(cmd):
    t0 = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    return cmd, r.returncode, r.stdout + r.stderr, time.time() - t0


def build(jobs: int | None = None, verbose: bool = False) -> str:
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    hip, cpp = sources()
    cmds, objs = [], []
    for f in hip:
        o = os.path.join(BUILD, f[:-4] + ".o")
        objs.append(o)
        cmds.append([hipcc, *COMMON, *DEVICE, "-c", os.path.join(CSRC, f), "-o", o])
    for f in cpp:
        o = os.path.join(BUILD, f[:-4] + ".o")
        objs.append(o)
        cmds.append([hipcc, *COMMON, "-c", os.path.join(CSRC, f), "-o", o])
    jobs = jobs or min(len(cmds), max(1, os.cpu_count() or 1))
    failed = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for cmd, rc, out, dt in ex.map(_compile, cmds):
            name = os.path.basename(cmd[-3])
            if rc != 0:
                failed.append((name, out))
            elif verbose:
                print(f"  compiled {name} in {dt:.1f}s", flush=True)
            if out.strip() and (verbose or rc != 0):
                print(out, file=sys.stderr)
    if failed:
        msg = "\n".join(f"--- {n}\n{o}" for n, o in failed)
        raise RuntimeError(f"HIP build failed:\n{msg}")
    tmp = LIB + ".tmp"
    link = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp, "-lpthread"]
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("-v", "--verbose", action="store_true")
    a = ap.parse_args()
    t0 = time.time()
    path = build(a.jobs, a.verbose)
    print(f"built {path} in {time.time() - t0:.1f}s")
