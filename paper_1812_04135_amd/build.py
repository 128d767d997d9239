"""Build the gfx950 RSST library in-tree with hipcc (no JIT, no torch extension).

    python -m paper_1812_04135_amd.build

writes paper_1812_04135_amd/librsst.so next to this file.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "librsst.so")
SOURCES = ["csrc/rsst_kernels.hip", "csrc/rsst_batch.hip", "csrc/rsst_adjoint.hip", "csrc/rsst_api.hip"]

# -packed-fp32-ops off: no packed FP32 instructions anywhere in the library
HIPFLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = (["hipcc"] + HIPFLAGS + ["-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(HERE, "csrc")]
           + [os.path.join(HERE, s) for s in SOURCES] + ["-o", tmp])
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
