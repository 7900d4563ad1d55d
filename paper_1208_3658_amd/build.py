"""Build libpc.so (gfx950) in-tree with hipcc.

Every translation unit is compiled with -ffp-contract=off: the binary64 steps
(unit vectors, edges, re-check, estimator) must round exactly as written, and
the binary32 kernel asks for its fused multiply-adds explicitly.  Packed FP32
instructions are disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpc.so")
SOURCES = ["pc_kernels.hip", "pc_prep.hip", "pc_api.cpp", "pc_tables.cpp", "pc_estimator.cpp", "pc_serve.cpp",
           "pc_tune.cpp", "pc_aperture.hip", "pc_kernels_t128.hip", "pc_prep_t128.hip", "pc_static.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False, defines=(), out: str = LIB) -> str:
    """Compile the library to `out`; `defines` are extra -D tuning macros
    (PC_R, PC_MAX_COLS, PC_JUNROLL, PC_WAVES_PER_EU)."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = out + ".tmp"
    cmd = [HIPCC, *FLAGS, *[f"-D{d}" for d in defines], "-I", os.path.join(os.path.dirname(HERE), "include"),
           *srcs, "-o", tmp, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass does not know the packed-fp32 feature name; that warning is harmless
    noise = ("packed-fp32-ops", "is not a recognized feature", "--hip-link")
    msgs = [l for l in (r.stdout + r.stderr).splitlines() if not any(n in l for n in noise)]
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs))
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
