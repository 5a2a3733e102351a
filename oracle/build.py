"""Build the CPU oracle shared library (test infrastructure).

The oracle is compiled with gcc at -O2, without fast-math and with
floating-point contraction off, so every expression rounds as written.
OpenMP parallelises the per-cell loops; it changes no result (each cell is
computed independently and the only reduction is a max).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, f) for f in ("mhd_oracle.c", "mhd_diffusion.c")]
LIB = os.path.join(HERE, "libmhd_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
        "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unknown-pragmas",
        *SRCS, "-o", LIB + ".tmp", "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
