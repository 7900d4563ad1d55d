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


def build(verbose: bool = False, out: str = LIB, opt=("-O2",)) -> str:
    """Builds the oracle into `out`; `opt` replaces the optimisation flags
    (tests build -O0, -march=native and sanitizer variants to check that the
    results do not depend on them)."""
    flags = [f for f in FLAGS if f != "-O2"]
    cmd = ["gcc", *opt, *flags, *SRCS, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
