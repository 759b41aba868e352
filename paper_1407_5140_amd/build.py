"""Build librewl.so (the HIP library) in-tree for gfx950."""
from __future__ import annotations

import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "librewl.so")
SOURCES = ["csrc/rewl_api.hip", "csrc/mlp.hip"]
DEPS = ["csrc/rewl_api.hip", "csrc/rewl_kernels.hip", "csrc/rewl_device.hpp", "csrc/mlp.hip",
        "csrc/ensemble_kernels.hip"]
HEADERS = ["rewl.h", "rewl_mlp.h"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-shared", "-fPIC", "-Wall",
    # FP expressions evaluate as written: the exact ln g arithmetic and the
    # double-double error-free transformations must not be fused implicitly
    "-ffp-contract=off",
    # no packed-FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the REWL library needs ROCm's hipcc to build")


def build_library(force: bool = True, verbose: bool = False) -> str:
    """Compile librewl.so; with force=False only when a source is newer."""
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(os.path.join(PKG, d)) for d in DEPS)
        for hdr in HEADERS:
            newest = max(newest, os.path.getmtime(os.path.join(ROOT, "include", hdr)))
        if os.path.getmtime(LIB) >= newest:
            return LIB
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + HIPCC_FLAGS + [os.path.join(PKG, s) for s in SOURCES] + ["-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(force=True))
