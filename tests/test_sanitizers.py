"""Host code under the sanitizers (CPU build, no GPU).

The library's host stages (validation, planner in every order including the
threaded paths, rank-local plans, halo plans) run under AddressSanitizer + UndefinedBehaviorSanitizer and under
ThreadSanitizer; the CPU oracle runs under AddressSanitizer +
UndefinedBehaviorSanitizer (its OpenMP runtime is not instrumented for
ThreadSanitizer).  Built with g++/gcc from the sources; no device code.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2609_04397_amd", "csrc")
HOST_SOURCES = [os.path.join(CSRC, f) for f in ("planner.cpp", "halo.cpp")]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")


def _build_and_run(tmp_path, name, cmd):
    exe = str(tmp_path / name)
    r = subprocess.run(cmd + ["-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               TSAN_OPTIONS="halt_on_error=1", OMP_NUM_THREADS="4")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "ERROR: " not in r.stderr, r.stderr[-4000:]
    return r.stdout


def _host_cmd(flags):
    return (["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__",
             "-I", "/opt/rocm/include", "-I", os.path.join(ROOT, "include")] + flags +
            [os.path.join(SAN, "host_driver.cpp")] + HOST_SOURCES + ["-lpthread"])


@pytest.mark.timeout(900)
def test_host_code_under_asan_ubsan(tmp_path):
    out = _build_and_run(tmp_path, "host_asan",
                         _host_cmd(["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]))
    assert "0 failed checks" in out


@pytest.mark.timeout(900)
def test_host_code_under_tsan(tmp_path):
    out = _build_and_run(tmp_path, "host_tsan", _host_cmd(["-fsanitize=thread"]))
    assert "0 failed checks" in out


@pytest.mark.timeout(600)
def test_oracle_under_asan_ubsan(tmp_path):
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(SAN, "oracle_driver.c"), os.path.join(ROOT, "oracle", "oracle.c"), "-lm"]
    out = _build_and_run(tmp_path, "oracle_asan", cmd)
    assert "oracle driver: rc 0" in out
