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
    """Compile every source to its own object (each carries the device code of
    the kernels it launches), all at once, then link the library. The device
    assembly the barrier-loop check reads is compiled alongside."""
    from concurrent.futures import ThreadPoolExecutor

    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    odir = os.path.join(HERE, "_build")
    os.makedirs(odir, exist_ok=True)
    objs = [os.path.join(odir, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    cflags = [f for f in FLAGS if f not in ("-shared", "-Wl,--no-undefined")]
    dev_flags = [f for f in cflags if f != "-fPIC"]
    jobs = [["hipcc", *cflags, "-c", src, "-o", obj] for src, obj in zip(srcs, objs)]
    if verbose:
        for cmd in jobs:
            print(" ".join(cmd), flush=True)

    def compile_obj(cmd):
        subprocess.run(cmd, check=True)

    def device_asm(src):
        return subprocess.run(["hipcc", *dev_flags, "--cuda-device-only", "-S", src, "-o", "-"],
                              check=True, capture_output=True, text=True).stdout

    with ThreadPoolExecutor(max_workers=min(2 * len(srcs), os.cpu_count() or 4)) as ex:
        futs = [ex.submit(compile_obj, cmd) for cmd in jobs]
        asms = [ex.submit(device_asm, src) for src in srcs] if check else []
        for f in futs:
            f.result()
        asm_txt = [f.result() for f in asms]
    link = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-Wl,--no-undefined", "-o", LIB + ".tmp", *objs]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    if check:
        from isa_check import check_asm
        bad = [b for txt in asm_txt for b in check_asm(txt)]
        if bad:
            os.remove(LIB + ".tmp")
            raise RuntimeError("barrier loop with a lane-divergent exit (would deadlock): " + ", ".join(bad))
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
