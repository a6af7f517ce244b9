"""Build the HIP library libskyline.so in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libskyline.so")
SOURCES = ["sky_api.hip", "sky_prims.hip", "sky_kernels.hip", "sky_dominance.hip", "sky_mlp.hip", "sky_batch.hip"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # comparisons and float64 partition arithmetic must be bit-reproducible
    "-ffp-contract=off",
    # no packed FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-Wno-unused-value",
    # every symbol the library uses must be defined in it
    "-Wl,--no-undefined",
]


def build(verbose: bool = False, check: bool = True) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    cmd = ["hipcc", *FLAGS, "-o", LIB + ".tmp", *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    if check:
        from isa_check import check_sources
        dev_flags = [f for f in FLAGS if f not in ("-fPIC", "-shared")]
        bad = check_sources(srcs, dev_flags)
        if bad:
            os.remove(LIB + ".tmp")
            raise RuntimeError("barrier loop with a lane-divergent exit (would deadlock): " + ", ".join(bad))
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
