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
SOURCES = ["csrc/rsst_kernels.hip", "csrc/rsst_batch.hip", "csrc/rsst_adjoint.hip", "csrc/rsst_adjoint_tile.hip",
           "csrc/rsst_api.hip"]
# the stage kernels, one object per dimension, storage type and addressing
# (big: 3D states of 2 GiB or more)
STAGE_UNITS = [(nd, st, 0) for nd in (3, 2, 1) for st in ("double", "float")] + \
              [(3, st, 1) for st in ("double", "float")]

# -packed-fp32-ops off: no packed FP32 instructions anywhere in the library
HIPFLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile each source to an object in _build/ (in parallel), then link.
    incremental: keep objects newer than every source and header."""
    from concurrent.futures import ThreadPoolExecutor

    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(HERE, "csrc")]
    compile_flags = [f for f in HIPFLAGS if f != "-shared"]
    objs, cmds = [], []
    for nd, st, big in STAGE_UNITS:
        obj = os.path.join(objdir, f"rsst_stage_{nd}d_{st}{'_big' if big else ''}.o")
        objs.append(obj)
        cmds.append(["hipcc"] + compile_flags + inc + [f"-DRSST_INST_NDIM={nd}", f"-DRSST_INST_ST={st}",
                                                        f"-DRSST_INST_BIG={big}", "-c",
                                                        os.path.join(HERE, "csrc/rsst_stage_inst.hip"), "-o", obj])
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.basename(src).replace(".hip", ".o"))
        objs.append(obj)
        cmds.append(["hipcc"] + compile_flags + inc + ["-c", os.path.join(HERE, src), "-o", obj])

    if incremental:
        hdr = max(os.path.getmtime(os.path.join(d, f)) for d in (os.path.join(HERE, "csrc"), os.path.join(ROOT, "include"))
                  for f in os.listdir(d) if f.endswith(".h"))
        stale = lambda c, o: (not os.path.exists(o) or
                              os.path.getmtime(o) < max(hdr, os.path.getmtime(os.path.join(HERE, c[-3]))))
        cmds = [c for c, o in zip(cmds, objs) if stale(c, o)]

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True, cwd=HERE)

    with ThreadPoolExecutor(max_workers=max(1, min(len(cmds), os.cpu_count() or 1))) as ex:
        list(ex.map(run, cmds))
    tmp = LIB + ".tmp"
    run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
