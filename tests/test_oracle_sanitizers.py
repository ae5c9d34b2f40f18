"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU): its
C source and a small driver (oracle_sanitize_main.c) are built with gcc's
sanitizers into a standalone executable that calls every lattice-level entry
point on small lattices with walls, solids, force fields, moving walls and
windows.  Any out-of-bounds access, use of freed memory or undefined operation
makes the run fail."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_runs_clean_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-static-libasan",
           os.path.join(ROOT, "oracle", "clbm_oracle.c"), os.path.join(HERE, "oracle_sanitize_main.c"),
           "-o", exe, "-lm"]
    build = subprocess.run(cmd, capture_output=True, text=True)
    if build.returncode != 0 and "asan" in build.stderr.lower():
        pytest.skip("the sanitizer runtime is not available: " + build.stderr[-300:])
    assert build.returncode == 0, build.stderr
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1:verify_asan_link_order=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stdout[-2000:] + run.stderr[-4000:]
    assert "oracle sanitizer run: ok" in run.stdout
