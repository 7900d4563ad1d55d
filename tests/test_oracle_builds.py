"""The oracle's results do not depend on how it is compiled: -O0, -O2 and
-O2 -march=native builds give the same bits (binary64 with contraction off,
so no fused multiply-add may creep in), and a build under AddressSanitizer
and UndefinedBehaviorSanitizer runs the same calls cleanly with the same
bits.  Each build runs in a child process (PC_ORACLE_LIB names it)."""
import os
import subprocess
import sys

import pytest

from oracle.build import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROBE = r"""
import hashlib
import numpy as np
import oracle, synth
h = hashlib.sha256()
x = np.concatenate([np.arange(-720.0, 720.5, 0.5), np.random.default_rng(3).uniform(-1e4, 1e4, 2000)])
for v in x:
    h.update(np.array(oracle.sincosd(float(v))).tobytes())
rng = np.random.default_rng(5)
patch = synth.centred_patch(20.0)
D = synth.neyman_scott(20, 10, 0.5, patch, rng)
R = synth.uniform_patch(300, patch, rng)
h.update(oracle.unit_vectors(*D).tobytes())
for e in (synth.log_edges(0.01, 10.0, 30), np.linspace(0.0, 180.0, 19)):
    h.update(oracle.chord2_edges(e).tobytes())
    dd, dr, rr = oracle.count(D, e), oracle.count(D, e, B=R, auto=False), oracle.count(R, e)
    for c in (dd, dr, rr):
        h.update(c.tobytes())
    h.update(oracle.wtheta(dd[1:-1], dr[1:-1], rr[1:-1], D[0].size, R[0].size).tobytes())
cat, side = synth.shear_catalog(3000, config=9)
m = oracle.aperture_grid(cat, (0.1, -0.2, side / 13.0, side / 11.0, 13, 11), 2.5, 35.0)
for k in ("map", "snr", "n_in", "s1", "s2", "qe_abs"):
    h.update(np.asarray(m[k]).tobytes())
print(h.hexdigest())
"""


def _run(lib_path, preload=None):
    env = dict(os.environ, PC_ORACLE_LIB=lib_path, OMP_NUM_THREADS="2",
               PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
    if preload:
        env["LD_PRELOAD"] = preload
        env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
        env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    p = subprocess.run([sys.executable, "-c", PROBE], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    assert p.returncode == 0, p.stderr[-3000:]
    assert "runtime error" not in p.stderr, p.stderr[-3000:]
    return p.stdout.strip()


def test_results_independent_of_optimisation_flags(tmp_path):
    ref = _run(build(out=str(tmp_path / "o2.so")))
    assert len(ref) == 64
    assert _run(build(out=str(tmp_path / "o0.so"), opt=("-O0",))) == ref
    assert _run(build(out=str(tmp_path / "native.so"), opt=("-O2", "-march=native"))) == ref


def test_sanitizer_build_runs_clean_with_the_same_bits(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    ref = _run(build(out=str(tmp_path / "o2.so")))
    lib = build(out=str(tmp_path / "san.so"),
                opt=("-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                     "-fno-sanitize-recover=all"))
    assert _run(lib, preload=asan) == ref
