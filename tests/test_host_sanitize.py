"""Host code under AddressSanitizer + UBSan, and under ThreadSanitizer (no GPU): builds the solver's
host-side sources (ingestion, presolve, BDD compiler, packer) with g++ and the
sanitizers into a driver that runs them on generated ILPs and batches."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2111_10270_amd", "csrc")


def build_and_run(tmp_path, name, sanitize, env):
    exe = str(tmp_path / name)
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-pthread", sanitize,
           "-fno-sanitize-recover=all", "-I", CSRC,
           os.path.join(CSRC, "problem.cpp"), os.path.join(ROOT, "tests", "host_sanitize.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, timeout=600)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=900, env=dict(os.environ, **env))
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "0 failures" in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_code_under_sanitizers(tmp_path):
    build_and_run(tmp_path, "host_asan", "-fsanitize=address,undefined",
                  {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=1", "UBSAN_OPTIONS": "print_stacktrace=1"})


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_threads_under_thread_sanitizer(tmp_path):
    """the threaded ingestion, compilation, packing and batch merge without
    data races (the same driver, built with ThreadSanitizer)"""
    build_and_run(tmp_path, "host_tsan", "-fsanitize=thread", {"TSAN_OPTIONS": "halt_on_error=1"})
