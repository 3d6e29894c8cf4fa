"""Builds libgsgp.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2106_04034_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgsgp.so")
PROBE = os.path.join(HERE, "copy_probe")
ARCH = os.environ.get("GSGP_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    # match the method's per-element arithmetic operation by operation
    "-ffp-contract=off",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]
# Per translation unit: the interpreter dispatches every op on wave-uniform
# op bits, and branch regions with uniform conditions keep plain scalar
# branches there (structurized as if divergent, every test costs a vector
# compare and exec masking); the other kernels are built without it (it
# made the variation kernel about 0.5 % slower).
UNIT_FLAGS = {
    "interp.hip": ["-mllvm", "-structurizecfg-skip-uniform-regions=true"],
}
SOURCES = ["kernels.hip", "interp.hip", "runtime.hip"]
BUILD_DIR = os.path.join(HERE, "_build")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the packed-fp32 feature and says so
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in res.stderr.splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{err}")
    if verbose and err.strip():
        print(err, file=sys.stderr)


def build(verbose: bool = False) -> str:
    """Compiles every source to an object of its own (so each can carry its
    own flags) and links libgsgp.so."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
        _run(["hipcc", f"--offload-arch={ARCH}", *FLAGS, *UNIT_FLAGS.get(src, []), "-c",
              os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    tmp = LIB + ".tmp"
    # every symbol resolved at link time (a missing definition fails the build)
    _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Wl,--no-undefined", "-o", tmp, *objs], verbose)
    os.replace(tmp, LIB)
    return LIB


def build_probe(verbose: bool = False) -> str:
    """Copy kernel of known size that calibrates the HBM byte counters."""
    tmp = PROBE + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-o", tmp, os.path.join(CSRC, "copy_probe.hip")]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{res.stderr}")
    os.replace(tmp, PROBE)
    return PROBE


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_probe(verbose=True))
