"""libpc's host code under sanitizers, on the CPU: the w(theta) server
(worker threads, admission, request parts, cancellation, queueing deadline,
patch replacement, launches that fail for lack of device memory), the edge
tables and guard bands, the estimators, the tuner's file parser and the
request planner are built with g++ together with a CPU fake of the device
layer (tests/sanitize/fake_device.cpp) and driven by
tests/sanitize/host_driver.cpp under AddressSanitizer + LeakSanitizer +
UndefinedBehaviorSanitizer, and under ThreadSanitizer."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1208_3658_amd", "csrc")
HOST_SOURCES = [os.path.join(CSRC, f) for f in ("pc_serve.cpp", "pc_tables.cpp", "pc_estimator.cpp", "pc_tune.cpp")]
HARNESS = [os.path.join(ROOT, "tests", "sanitize", f) for f in ("fake_device.cpp", "host_driver.cpp")]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                                reason="needs g++ and the ROCm headers")


def _build_and_run(tmp_path, flags, env_extra):
    exe = str(tmp_path / "host_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *flags, "-D__HIP_PLATFORM_AMD__",
           "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"), *HOST_SOURCES, *HARNESS, "-o", exe,
           "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, **env_extra)
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    return r.returncode, out


def test_host_code_under_address_leak_and_undefined_behaviour_sanitizers(tmp_path):
    rc, out = _build_and_run(tmp_path, ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
                             {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0",
                              "UBSAN_OPTIONS": "print_stacktrace=1"})
    assert "ERROR: AddressSanitizer" not in out, out[-6000:]
    assert "ERROR: LeakSanitizer" not in out, out[-6000:]
    assert "runtime error" not in out, out[-6000:]
    assert rc == 0 and "0 check(s) failed" in out, out[-6000:]
    assert "finished" in out


def test_host_code_under_thread_sanitizer(tmp_path):
    rc, out = _build_and_run(tmp_path, ["-fsanitize=thread"], {"TSAN_OPTIONS": "halt_on_error=0:second_deadlock_stack=1"})
    assert "WARNING: ThreadSanitizer" not in out, out[-8000:]
    assert rc == 0 and "0 check(s) failed" in out, out[-6000:]
