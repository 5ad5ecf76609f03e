"""Build libpi.so (the C-ABI HIP library) in-tree for gfx950.

    python -m paper_2406_16091_amd.build

Compiles every ``csrc/*.hip`` with hipcc for gfx950 only (one object per
source, in parallel, under ``_build/``) and links them into
``paper_2406_16091_amd/libpi.so``.  Flags:
  * ``-ffp-contract=off``: no implicit FMA contraction; every FMA in the
    kernels is written out, so float32 results are exactly what the source
    says (the binning's cell decision and the cutoff filter rely on this);
  * ``-target-feature -packed-fp32-ops``: no packed FP32 instructions.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpi.so")
OBJ = os.path.join(os.path.dirname(HERE), "_build")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _quiet(stderr: str) -> str:
    return "\n".join(ln for ln in (stderr or "").splitlines()
                     if "packed-fp32-ops" not in ln and ln.strip())


def _compile(src: str) -> tuple[str, subprocess.CompletedProcess]:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    r = subprocess.run([HIPCC, *FLAGS, "-c", src, "-o", obj], capture_output=True, text=True)
    return obj, r


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    if verbose:
        print(f"{HIPCC} {' '.join(FLAGS)} -c <src> for {len(srcs)} sources", flush=True)
    jobs = min(len(srcs), max(1, min(os.cpu_count() or 1, 16)))
    objs, failed = [], False
    with cf.ThreadPoolExecutor(jobs) as ex:
        for src, (obj, r) in zip(srcs, ex.map(_compile, srcs)):
            objs.append(obj)
            if r.returncode != 0:
                failed = True
                sys.stderr.write(f"--- {src}\n{r.stdout}{r.stderr}")
            elif verbose and _quiet(r.stderr):
                sys.stderr.write(_quiet(r.stderr) + "\n")
    if failed:
        raise RuntimeError("hipcc failed compiling libpi.so sources")
    tmp = LIB + ".tmp"
    r = subprocess.run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed linking libpi.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
