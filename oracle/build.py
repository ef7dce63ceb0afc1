"""Compile the CPU oracle (test infrastructure) into two shared libraries.

``liboracle.so`` is the double-precision oracle; ``liboracle_f32.so`` is its
single-precision twin, used only to size single-precision tolerances.  Both
also export the interface's lb_* entry points on host memory
(oracle_abi.c), so a test can drive either library with one call sequence.  Plain
gcc, OpenMP over lattice rows, no floating-point contraction so the rounding
of every expression is the one written in the source.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "oracle.c"), os.path.join(HERE, "oracle_abi.c")]
TARGETS = {
    "liboracle.so": [],
    "liboracle_f32.so": ["-DORACLE_F32"],
}


def build(verbose=False):
    for name, extra in TARGETS.items():
        out = os.path.join(HERE, name)
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-fPIC", "-shared", "-Wall", "-Wextra",
               *extra, *SRCS, "-o", out + ".tmp", "-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


if __name__ == "__main__":
    build(verbose=True)
