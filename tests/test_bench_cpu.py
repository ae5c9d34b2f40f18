"""The benchmark's host-side definitions (CPU): the algorithmic bytes per node update each roofline
fraction is computed from, the refusal of more than one GPU, and the rule that a counter summary is
only used when it was taken on the current kernel source."""
from __future__ import annotations

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("storage,field,solid,q,expected", [
    ("f32", True, False, 27, 228),   # the 512^3 Kolmogorov headline: 2 x 27 x 4 + 3 x 4
    ("f32", False, False, 27, 216),  # Taylor-Green, cavity: no force field
    ("f64", True, False, 27, 456),
    ("f16", True, False, 27, 120),
    ("bf16", True, False, 27, 120),
    ("f32", True, False, 19, 164),   # D3Q19 (Appendix A)
    ("f64", True, False, 19, 328),
    ("f16", True, False, 19, 88),
    ("f32", False, True, 27, 217),   # per fluid node of the porous duct, plus the 1-byte mask
])
def test_algorithmic_bytes_per_node_update(storage, field, solid, q, expected):
    assert bench.bytes_per_node(storage, field, solid, q) == expected


def test_adjoint_bytes_per_node():
    """State 27 x 4 read, lambda 27 x 4 read and written, dJ/dF 3 x 4 read and written, force field
    3 x 4 read, mask 1 byte; with FP64 storage every one of these but the mask in 8-byte words."""
    assert bench.ADJ_BYTES == 108 + 216 + 24 + 12 + 1 == 361
    assert bench.ADJ_BYTES_F64 == 216 + 432 + 48 + 24 + 1 == 721


def test_more_than_one_gpu_is_refused():
    run = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert run.returncode != 0
    assert "one GPU" in run.stdout + run.stderr


def test_counter_summary_is_used_only_for_the_kernel_source_it_was_taken_on(tmp_path):
    pmc = {"kernel_src_sha": bench.kernel_sha(), "size": 512, "fused": True, "hbm_bytes_per_launch": 1.5e10}
    path = tmp_path / "pmc.json"
    path.write_text(json.dumps(pmc))
    assert bench.pmc_traffic(str(path), 512, True) == 1.5e10
    assert bench.pmc_traffic(str(path), 256, True) is None      # another lattice
    assert bench.pmc_traffic(str(path), 512, False) is None     # another launch kind
    pmc["kernel_src_sha"] = "0" * 16
    path.write_text(json.dumps(pmc))
    assert bench.pmc_traffic(str(path), 512, True) is None      # kernels changed since
    assert bench.pmc_traffic(str(tmp_path / "missing.json"), 512, True) is None
