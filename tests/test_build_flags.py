"""The device code of the built library contains no packed FP32 vector instructions.

build.py passes the feature flag that keeps the compiler from forming them.  The host pass of hipcc
does not know the feature and says it ignores it; this test checks, on the CPU, that the device pass
honours it: it extracts the gfx950 code object from libclbm.so and disassembles it.
"""
from __future__ import annotations

import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1801_04586_amd", "libclbm.so")
LLVM = "/opt/rocm/llvm/bin"
PACKED_FP32 = re.compile(r"\bv_pk_(add|mul|fma)_f32\b")


@pytest.mark.skipif(not os.path.exists(LIB), reason="libclbm.so is not built")
@pytest.mark.skipif(not os.path.exists(os.path.join(LLVM, "clang-offload-bundler")), reason="no LLVM tools")
def test_device_code_has_no_packed_fp32_instructions(tmp_path):
    fat = tmp_path / "fatbin"
    co = tmp_path / "gfx950.co"
    subprocess.run([f"{LLVM}/llvm-objcopy", f"--dump-section=.hip_fatbin={fat}", LIB, str(tmp_path / "ignored")],
                   check=True)
    subprocess.run([f"{LLVM}/clang-offload-bundler", "--unbundle", "--type=o",
                    "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--input={fat}", f"--output={co}"], check=True)
    asm = subprocess.run([f"{LLVM}/llvm-objdump", "-d", str(co)], check=True, capture_output=True, text=True).stdout
    assert "k_step2" in asm and "k_adjoint" in asm  # the kernels are there
    found = PACKED_FP32.findall(asm)
    assert not found, f"{len(found)} packed FP32 instructions in the device code"
