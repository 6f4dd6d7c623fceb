"""The serving scheduler (csrc/serve_policy.hpp) on the CPU: the host test
in tests/host/serve_policy_test.cpp drives it with a stub executor (three
worker threads in place of the device streams) and is built with g++ three
ways: plain, under ThreadSanitizer, and under AddressSanitizer with
UndefinedBehaviorSanitizer.  No GPU and no HIP are involved."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "host", "serve_policy_test.cpp")
GXX = shutil.which("g++")


def _build_and_run(tmp_path, name, flags, env=None):
    exe = str(tmp_path / name)
    cmd = [GXX, "-std=c++17", "-O1", "-g", "-pthread", *flags, SRC, "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    run_env = dict(os.environ)
    run_env.update(env or {})
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=run_env)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "all scenarios passed" in out.stdout
    return out


@pytest.mark.skipif(GXX is None, reason="g++ not found")
def test_policy_plain(tmp_path):
    _build_and_run(tmp_path, "plain", [])


@pytest.mark.skipif(GXX is None, reason="g++ not found")
def test_policy_thread_sanitizer(tmp_path):
    out = _build_and_run(tmp_path, "tsan", ["-fsanitize=thread"], {"TSAN_OPTIONS": "halt_on_error=1"})
    assert "ThreadSanitizer" not in out.stderr


@pytest.mark.skipif(GXX is None, reason="g++ not found")
def test_policy_address_sanitizer(tmp_path):
    out = _build_and_run(tmp_path, "asan", ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
                         {"ASAN_OPTIONS": "detect_leaks=1"})
    assert "AddressSanitizer" not in out.stderr
