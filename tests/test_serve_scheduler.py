"""CPU tests of the serving scheduler (continuous batching, memory admission,
FIFO, failure handling) with a fake executor, built with g++ under
ThreadSanitizer. No GPU involved."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


CLANG = "/opt/rocm/llvm/bin/clang++"


def _build_and_run(extra, cxx="g++"):
    src = [os.path.join(ROOT, "tests", "serve_sched_test.cpp"),
           os.path.join(ROOT, "paper_1810_03099_amd", "csrc", "serve_core.cpp")]
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "sched")
        subprocess.check_call([cxx, "-std=c++17", "-O1", "-g", *extra, *src, "-o", exe, "-lpthread"])
        r = subprocess.run([exe], capture_output=True, text=True, timeout=240,
                           env={**os.environ, "TSAN_OPTIONS": "halt_on_error=1"})
    return r


def test_scheduler_plain():
    r = _build_and_run([])
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ALL OK" in r.stdout


def test_scheduler_under_thread_sanitizer():
    # clang's runtime: GCC 11's ThreadSanitizer does not intercept the
    # pthread_cond_clockwait that std::condition_variable::wait_for uses and
    # reports a false double lock.
    if not os.path.exists(CLANG):
        pytest.skip("clang++ not available")
    r = _build_and_run(["-fsanitize=thread"], cxx=CLANG)
    if r.returncode != 0 and "FATAL: ThreadSanitizer: unexpected memory mapping" in r.stderr:
        pytest.skip("ThreadSanitizer cannot run in this environment")
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ALL OK" in r.stdout and "WARNING: ThreadSanitizer" not in r.stderr
