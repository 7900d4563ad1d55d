"""Compile the CPU oracle into oracle/libpc_oracle.so (test infrastructure):
pair counting (pc_oracle.c) and aperture-mass maps (ap_oracle.c).

Flags: binary64 throughout, no fused multiply-add (-ffp-contract=off; GCC's
default for GNU C would contract), no fast-math, SSE2 arithmetic (x86-64
default), OpenMP over rows.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "pc_oracle.c"), os.path.join(HERE, "ap_oracle.c")]
LIB = os.path.join(HERE, "libpc_oracle.so")

FLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
         "-ffp-contract=off", "-fno-fast-math", "-fno-unsafe-math-optimizations"]


def build(verbose: bool = False) -> str:
    cmd = ["gcc", *FLAGS, *SRCS, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
