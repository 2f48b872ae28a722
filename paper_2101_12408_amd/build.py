"""Builds libmpm.so (HIP kernels for gfx950 + host library + host sampler) in-tree.

    python -m paper_2101_12408_amd.build

hipcc cross-compiles for gfx950 without a GPU.  Packed FP32 instructions are disabled
(-packed-fp32-ops target feature), the compiler still vectorises everything else.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmpm.so")
ARCH = os.environ.get("MPM_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose=False):
    srcs = [os.path.join(CSRC, "mpm.hip"), os.path.join(CSRC, "sampler.cpp"), os.path.join(CSRC, "serve.cpp")]
    tmp = OUT + ".tmp"
    cmd = [hipcc(), "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-result", "-Wno-unknown-warning-option",
           "-I", os.path.join(HERE, "..", "include"),
           *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
