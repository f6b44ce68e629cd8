"""The serving scheduler (paper_2308_09782_amd/csrc/server_core.h) on the host,
against a stub engine, under the thread sanitizer and under the address and
undefined-behaviour sanitizers (tests/native/server_sched_check.cpp).  No GPU:
this checks the scheduling logic itself - admission by footprint, the
initialisation worker, chunked stepping, failure paths - for data races,
memory errors and leaks."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "native", "server_sched_check.cpp")


def _build_and_run(tmp_path, flags, env_extra):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-pthread", *flags,
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2308_09782_amd", "csrc"),
           SRC, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, **env_extra)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "OK" in out.stdout
    assert "WARNING: ThreadSanitizer" not in out.stderr, out.stderr
    return out


def test_scheduler_under_thread_sanitizer(tmp_path):
    _build_and_run(tmp_path, ["-fsanitize=thread"], {"TSAN_OPTIONS": "halt_on_error=1"})


def test_scheduler_under_address_and_undefined_sanitizers(tmp_path):
    _build_and_run(tmp_path, ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
                   {"ASAN_OPTIONS": "detect_leaks=1"})
