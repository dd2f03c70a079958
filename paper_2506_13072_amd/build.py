"""Build libvflb.so for gfx950 with hipcc (in-tree, next to this file)."""
from __future__ import annotations

import os
import subprocess

import hashlib

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libvflb.so")
CSRC = os.path.join(HERE, "csrc")
SOURCES = [os.path.join(CSRC, "vflb.hip"), os.path.join(CSRC, "mlp.hip")]
HEADER = os.path.join(os.path.dirname(HERE), "include", "vflb.h")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no fused multiply-add contraction: every instantiation (tile shape,
    # batched or single) rounds the same way, so results are bitwise
    # independent of launch configuration; measured no slower (memory-bound)
    "-ffp-contract=off",
    "-Wall", "-Wno-unused-function",
]


# device code each step kernel is compiled from
KERNEL_FILES = {
    "step2d": ("step2d.h", "kernels.h", "layout.h", "lattice.h"),
    "step3d": ("step3d.h", "kernels.h", "layout.h", "lattice.h"),
    "aa3d": ("aa3d.h", "kernels.h", "layout.h", "lattice.h"),
}


def kernel_sources_sha(kernel: str) -> str:
    """SHA-256 over what one step kernel is compiled from (its device
    headers and the compiler flags).
    Recorded next to measured hardware counters, so a consumer can tell
    whether the counters still describe the kernel it runs."""
    h = hashlib.sha256()
    paths = [os.path.join(CSRC, n) for n in KERNEL_FILES[kernel]]
    for path in paths:
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(HIPCC_FLAGS).encode())
    return h.hexdigest()


def build(verbose: bool = False) -> str:
    """Compile the HIP library (always recompiles); returns its path."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-o", tmp, *SOURCES]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
