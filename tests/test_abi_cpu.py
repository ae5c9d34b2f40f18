"""C-ABI checks that need no GPU: the library loads, exports every entry point
that include/clbm.h declares, and rejects bad arguments on the host before
any HIP call."""
from __future__ import annotations

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "clbm.h")


def _lib():
    from paper_1801_04586_amd import clbm

    if not os.path.exists(clbm.LIB_PATH):
        from paper_1801_04586_amd import build

        build.build()
    return clbm.load_library()


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(clbm_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_abi():
    names = _declared_functions()
    for required in ("clbm_create", "clbm_init", "clbm_step", "clbm_run", "clbm_moments", "clbm_adjoint_step",
                     "clbm_loss_seed", "clbm_destroy", "clbm_strerror", "clbm_get_populations",
                     "clbm_set_populations", "clbm_copy", "clbm_set_rates", "clbm_set_force"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1801_04586_amd import clbm

    _lib()
    out = subprocess.run(["nm", "-D", "--defined-only", clbm.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (clbm_[a-z_0-9]+)", out))
    missing = [n for n in _declared_functions() if n not in exported]
    assert not missing, missing


def test_desc_layout_matches_header():
    from paper_1801_04586_amd.clbm import Desc

    assert ctypes.sizeof(Desc) == 320
    assert Desc.s.offset == 32 and Desc.force.offset == 144 and Desc.solid.offset == 152
    assert Desc.collision.offset == 160 and Desc.wall_velocity.offset == 168 and Desc.plane_stride.offset == 312


def test_default_plane_stride():
    """N rounded up to 256 bytes plus 4 KiB, in elements of the storage type; -1 for bad input."""
    L = _lib()
    assert L.clbm_default_plane_stride(512, 512, 512, 1) == 512 ** 3 + 1024
    assert L.clbm_default_plane_stride(7, 6, 5, 0) == 224 + 512
    assert L.clbm_default_plane_stride(7, 6, 5, 2) == 256 + 2048
    assert L.clbm_default_plane_stride(0, 6, 5, 1) == -1
    assert L.clbm_default_plane_stride(4, 4, 4, 9) == -1
    assert L.clbm_default_plane_stride(2048, 2048, 1024, 1) == -1
    # products that overflow 64 bits (2^90 wraps to 0) are rejected, not wrapped
    assert L.clbm_default_plane_stride(1 << 30, 1 << 30, 1 << 30, 1) == -1
    assert L.clbm_default_plane_stride(1 << 30, 1 << 30, 16, 1) == -1


def test_strerror_and_version():
    from paper_1801_04586_amd import clbm

    L = _lib()
    declared = int(re.search(r"#define CLBM_ABI_VERSION (\d+)", open(HEADER).read()).group(1))
    assert L.clbm_abi_version() == declared == clbm.ABI_VERSION
    for code, word in [(0, b"success"), (1, b"invalid"), (2, b"rate"), (3, b"storage"), (4, b"HIP"),
                       (5, b"non-finite")]:
        assert word in L.clbm_strerror(code)
    assert L.clbm_strerror(99) == b"unknown status"
    assert L.clbm_last_error(None) is not None


def _create(desc):
    from paper_1801_04586_amd.clbm import load_library

    L = load_library()
    h = ctypes.c_void_p(123)
    rc = L.clbm_create(ctypes.byref(h), ctypes.byref(desc) if desc is not None else None, None)
    return rc, h, L.clbm_last_error(None).decode()


def _desc(**kw):
    from paper_1801_04586_amd.clbm import make_desc

    args = dict(dims=(4, 4, 4), walls=(0, 1, 0), storage="f32", rates=[1.0, 1.0, 1.5] + [1.0] * 7)
    args.update(kw)
    return make_desc(**args)


@pytest.mark.parametrize("kw,code,word", [
    (dict(dims=(0, 4, 4)), 1, "dims"),
    (dict(dims=(2048, 2048, 1024)), 1, "2^31"),
    (dict(dims=(1 << 30, 1 << 30, 1 << 30), plane_stride=0), 1, "2^31"),
    (dict(dims=(1 << 21, 1 << 21, 1 << 22), plane_stride=0), 1, "2^31"),
    (dict(walls=(0, 2, 0)), 1, "wall"),
    (dict(rates=[1.0, 1.0, 2.0] + [1.0] * 7), 2, "s2"),
    (dict(rates=[1.0, 1.0, 1.5, 1.0, 0.0] + [1.0] * 5), 2, "s3"),
    (dict(rates=[1.0] * 9 + [float("nan")]), 2, "s6"),
    (dict(force=(0.0, float("inf"), 0.0)), 1, "force"),
    (dict(collision="mrt", lattice="d3q19"), 1, "MRT"),
    (dict(wall_velocity={(0, 1): (0.1, 0.0, 0.0)}), 1, "periodic"),
    (dict(wall_velocity={(1, 1): (float("nan"), 0.0, 0.0)}), 1, "wall velocity"),
    (dict(plane_stride=63), 1, "plane_stride"),
    (dict(dims=(1024, 1024, 513), storage="f64"), 1, "too large"),
    (dict(dims=(1024, 1024, 1025), storage="f16"), 1, "too large"),
    (dict(plane_stride=66), 1, "16 bytes"),
])
def test_create_rejects_bad_descriptions_before_any_hip_call(kw, code, word):
    rc, h, msg = _create(_desc(**kw))
    assert rc == code and h.value is None and word in msg


def test_create_rejects_bad_storage_and_lattice():
    d = _desc()
    d.storage = 7
    assert _create(d)[0] == 3
    for lat in (2, -1):
        d = _desc()
        d.lattice = lat
        rc, h, msg = _create(d)
        assert rc == 1 and h.value is None and "lattice" in msg
    d = _desc()
    d.collision = 5
    assert _create(d)[0] == 1
    d = _desc()
    d.reserved = 1
    assert _create(d)[0] == 1
    assert _create(None)[0] == 1


def test_calls_on_null_context_fail_cleanly():
    L = _lib()
    assert L.clbm_step(None, None, None) == 1
    assert L.clbm_run(None, None, None, 3, None) == 1
    assert L.clbm_set_options(None, 0) == 1
    assert L.clbm_fused_pairs(None) == 1
    assert L.clbm_moments(None, None, None, None, None, None) == 1
    assert L.clbm_adjoint_step(None, None, None, None, None, None) == 1
    assert L.clbm_trajectory(None, None, None, 2) == 1
    assert L.clbm_destroy(None) == 0
    assert L.clbm_set_rates(None, None) == 1


def test_fastdiv_formula_on_host():
    """The node-index division by multiply-shift used in the kernels (31-bit numerators)."""
    for d in (1, 2, 3, 5, 7, 16, 31, 100, 101, 320, 512, 640, 1000, 65535, 131071, 2 ** 20 + 7):
        l = 0
        while (1 << l) < d:
            l += 1
        shift = 31 + l
        mul = (1 << shift) // d + 1
        rng = np.random.default_rng(d)
        ns = np.concatenate([rng.integers(0, 2 ** 31 - 1, 2000), np.arange(0, min(3 * d + 3, 4000)),
                             d * rng.integers(0, (2 ** 31 - 1) // d, 500) + rng.integers(-1, 2, 500) % d,
                             [2 ** 31 - 1]])
        for n in ns.tolist():
            assert (n * mul) >> shift == n // d
