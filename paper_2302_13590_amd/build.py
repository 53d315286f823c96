"""Build libpt.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2302_13590_amd.build
    python -m paper_2302_13590_amd.build --src DIR --out PATH   # a library from another copy of csrc/
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpt.so")
SOURCES = ["pt_kernels.hip", "pt_api.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # the FP64 path must round exactly as written: no FMA contraction, no fast math
    "-ffp-contract=off",
    "-fno-fast-math",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-result",
]


def build(verbose: bool = False, src: str = CSRC, out: str = LIB) -> str:
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-I", INCLUDE, "-o", tmp] + [os.path.join(src, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--src", default=CSRC, help="directory holding pt_kernels.hip and pt_api.hip")
    ap.add_argument("--out", default=LIB)
    a = ap.parse_args()
    print(build(verbose=True, src=os.path.abspath(a.src), out=os.path.abspath(a.out)))
    sys.exit(0)
