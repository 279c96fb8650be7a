"""Build libp2r.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
SO = os.path.join(HERE, "libp2r.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # matrix-core accumulators in the VGPRs: with the AGPR form the learned
    # fit kernel held 232 VGPRs + 48 AGPRs of the unified 512 (one wave per
    # SIMD) and copied every accumulator out of the AGPRs; in VGPR form it
    # needs 196 (two waves per SIMD) and no copies
    "-mllvm", "-amdgpu-mfma-vgpr-form=1",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]
SOURCES = ["kernels.hip", "ragged.hip", "mlp.hip", "capi.cpp"]


def source_hash() -> str:
    """Hash of every source the library is compiled from (the C ABI header
    included).  It is compiled into the library's version string, which keys
    the autotuner's cache: a rebuilt kernel is timed again, never served a
    choice made for other code."""
    h = hashlib.sha256()
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp", ".h")))
    for f in files:
        h.update(f.encode())
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(ROOT, "include", "p2r.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    cmd = [HIPCC, *FLAGS, f"-DP2R_SRC_HASH=\"{source_hash()}\"", "-I", os.path.join(ROOT, "include"),
           "-x", "hip", *srcs, "-o", SO + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(SO + ".tmp", SO)
    return SO


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
