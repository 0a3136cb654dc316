"""Compile the HIP library (libhelm.so) for gfx950, in place.

    python -m paper_2608_22946_amd.build

Each source compiles to its own object (in parallel, under _build/ beside this
file); the objects are then linked into libhelm.so.  Every kernel is launched
from the translation unit that defines it, so no relocatable device code is
needed.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libhelm.so")
OBJ_DIR = os.path.join(HERE, "_build")
SOURCES = ["stencil.hip", "stencil_mixed.hip", "transfer.hip", "vector.hip", "adjoint.hip", "helm.hip", "noalloc.hip"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep hand-written float code off the packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def build(verbose=False, jobs=None):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ_DIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(HERE, "csrc", s))]
    objs = [os.path.join(OBJ_DIR, os.path.splitext(s)[0] + ".o") for s in srcs]

    def compile_one(i):
        cmd = [hipcc] + FLAGS + inc + ["-c", os.path.join(HERE, "csrc", srcs[i]), "-o", objs[i]]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)

    with ThreadPoolExecutor(max_workers=jobs or min(len(srcs), os.cpu_count() or 1)) as ex:
        list(ex.map(compile_one, range(len(srcs))))
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
