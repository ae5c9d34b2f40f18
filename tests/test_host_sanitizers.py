"""The library's GPU-free host logic (descriptor and rate checks, plane stride, status strings, the
z-chunking of the fused launch: paper_1801_04586_amd/csrc/host_logic.hpp, which clbm.hip includes)
built with g++ under AddressSanitizer and UndefinedBehaviorSanitizer and run on the CPU by a driver
(host_sanitize_main.cpp) that feeds it every kind of invalid descriptor and a sweep of launch shapes."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_host_logic_runs_clean_under_asan_and_ubsan(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "host_sanitize")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-static-libasan", "-Wall", "-Wextra",
           os.path.join(HERE, "host_sanitize_main.cpp"), "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True)
    if build.returncode != 0 and "asan" in build.stderr.lower():
        pytest.skip("the sanitizer runtime is not available: " + build.stderr[-300:])
    assert build.returncode == 0, build.stderr
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1:verify_asan_link_order=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert run.returncode == 0, run.stdout[-2000:] + run.stderr[-4000:]
    assert "host sanitizer run: ok" in run.stdout
