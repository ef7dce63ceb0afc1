"""Build liblb.so (the HIP library behind include/lb.h) for gfx950.

Compiles in-tree with hipcc; the result sits next to this file and is what
the Python binding loads.  Usage: ``python -m paper_1008_2865_amd.build``.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "liblb.so")
SOURCES = [os.path.join(HERE, "csrc", "lb_kernels.hip"),
           os.path.join(HERE, "csrc", "lb_adjoint.hip"),
           os.path.join(HERE, "csrc", "lb_structure.hip"),
           os.path.join(HERE, "csrc", "lb_noalloc.hip"),
           os.path.join(HERE, "csrc", "lb_api.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # Packed-FP32 instructions stay off: the compiler must not form them.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"),
    "-I", os.path.join(HERE, "csrc"),
]


def build(verbose=False, extra=()):
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, *extra, *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
