"""Build libfj.so (HIP for gfx950) in-tree with hipcc."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfj.so")
SOURCES = ["fj_plan.cpp", "fj_api.cpp", "fj_learn.cpp", "fj_bushy.cpp", "fj_kernels.hip", "fj_batch.hip", "fj_learn.hip",
           "fj_noalloc.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-value", "-Wno-unused-result",
    # keep the compiler away from packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False, defines=(), lib: str = LIB, bdir: str = None) -> str:
    objs = []
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    bdir = bdir or os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    for s in SOURCES:
        o = os.path.join(bdir, s + ".o")
        lang = ["-x", "hip"] if s.endswith(".hip") else []
        cmd = [HIPCC] + FLAGS + ["-D" + d for d in defines] + inc + lang + ["-c", os.path.join(CSRC, s), "-o", o]
        if verbose:
            print(" ".join(cmd))
        subprocess.check_call(cmd)
        objs.append(o)
    tmp = lib + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
