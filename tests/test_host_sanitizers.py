"""The library's host code under AddressSanitizer and ThreadSanitizer, on the CPU.

The host side of every translation unit is built without its device code and
linked with a stand-in for the HIP runtime (tests/hoststub/hip_stub.cpp) that
keeps device memory in host memory, queues asynchronous copies until something
waits for them, and reports copies whose host buffers change or die before
that wait, early reads of copy destinations, copies across streams that no
event orders, and copies of the wrong kind or out of bounds.  The driver runs
batched solves on 16 worker threads, single contexts from 16 threads, the
allocation-free entry point, and a sweep of injected HIP failures over a batched
solve (every error path must return an error, leave nothing queued and free
everything).  Canary runs plant each kind of mistake in the driver's own code
and require the harness to report it.
"""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "hoststub"))

pytestmark = pytest.mark.skipif(
    not (os.path.exists("/opt/rocm/bin/hipcc") and os.path.exists("/opt/rocm/llvm/bin/clang++")
         and shutil.which("nm")),
    reason="needs hipcc, clang++ and nm")

ENV = dict(os.environ, RPCA_BATCH_WORKERS="16",
           ASAN_OPTIONS="detect_stack_use_after_return=1:detect_leaks=1",
           TSAN_OPTIONS="halt_on_error=0")


@pytest.fixture(scope="module")
def drivers():
    import build as hoststub_build  # tests/hoststub/build.py
    return {san: hoststub_build.build(san) for san in ("address", "thread")}


def _run(exe, *args, timeout=600):
    res = subprocess.run([exe, *args], capture_output=True, text=True, env=ENV, timeout=timeout)
    return res.returncode, res.stdout + res.stderr


@pytest.mark.parametrize("san,points", [("address", 40), ("thread", 6)])
def test_library_host_code_clean(drivers, san, points):
    rc, out = _run(drivers[san], str(points))
    print(out[-2000:])
    assert "ERROR: AddressSanitizer" not in out
    assert "WARNING: ThreadSanitizer" not in out
    assert "stand-in problems 0, failed checks 0" in out
    assert f"failure sweep: {points} points" in out
    # every injected failure surfaced as an error of the solve
    assert f"{points} solves returned an error" in out
    assert rc == 0


@pytest.mark.parametrize("canary,san,expect", [
    ("freed-source", "address", "heap-use-after-free"),
    ("early-read", "address", "use-after-poison"),
    ("rewritten-source", "address", "host source of a queued copy changed"),
    ("cross-stream", "address", "no event orders them"),
    ("race", "thread", "WARNING: ThreadSanitizer: data race"),
])
def test_harness_reports_planted_mistakes(drivers, canary, san, expect):
    rc, out = _run(drivers[san], "--canary", canary, timeout=120)
    assert rc != 0, out[-2000:]
    assert expect in out, out[-2000:]
