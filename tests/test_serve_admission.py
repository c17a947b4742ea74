"""The serving core's admission under many threads, on the CPU: a mock device
drives the same queue, admission and thread code as the library's server
(paper_2607_12074_amd/csrc/m4_serve_core.h), built with a thread sanitizer.
Every request comes back once with its own result, requests beyond the
budget are refused, admission is first come first served, and the memory
the mock device holds never exceeds the budget."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "serve_mock", "mock_serve.cpp")


def _build(tmp_path, sanitize):
    exe = str(tmp_path / ("mock_serve_" + sanitize))
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", "-fsanitize=" + sanitize, SRC, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail("build failed:\n" + r.stderr[-3000:])
    return exe


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
@pytest.mark.parametrize("sanitize", ["thread", "address"])
def test_admission_under_threads(tmp_path, sanitize):
    exe = _build(tmp_path, sanitize)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 second_deadlock_stack=1",
               ASAN_OPTIONS="detect_leaks=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "OK" in r.stdout and "WARNING: ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
