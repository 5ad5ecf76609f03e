"""Build libpi.so (the C-ABI HIP library) in-tree for gfx950.

    python -m paper_2406_16091_amd.build

Compiles every ``csrc/*.hip`` with hipcc for gfx950 only and links them into
``paper_2406_16091_amd/libpi.so``.  Flags:
  * ``-ffp-contract=off``: no implicit FMA contraction; every FMA in the
    kernels is written out, so float32 results are exactly what the source
    says (the binning's cell decision and the cutoff filter rely on this);
  * ``-target-feature -packed-fp32-ops``: no packed FP32 instructions.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpi.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *sources()]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libpi.so")
    err = [ln for ln in (r.stderr or "").splitlines()
           if "packed-fp32-ops" not in ln and ln.strip()]
    if verbose and err:
        sys.stderr.write("\n".join(err) + "\n")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
