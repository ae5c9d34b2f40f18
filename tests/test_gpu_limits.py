"""Edge cases at the limits of the C ABI: the largest lattices the 32-bit plane
offsets allow (N = 2^30 nodes with FP16 storage and an FP32 force field;
N = 2^29 with FP64 storage, D3Q19), checked on sampled nodes near the last node
against the oracle on a window around them; and empty calls (zero steps, zero
samples)."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

RATES = np.array([1.0, 1.0, 1.6, 1.2, 1.3, 0.9, 1.1, 1.25, 0.95, 1.05])


def _free_bytes():
    torch.cuda.empty_cache()
    return torch.cuda.mem_get_info()[0]


def _window_check(lat, field_dev, dims, lattice, steps, centres, tol):
    """Oracle on a periodic 9^3 window around each centre, started from rest with the window's force field;
    the centre node is exact after `steps` <= 4 steps (light cone)."""
    nx, ny, nz = dims
    got = lat.sample(centres)
    for k, (x, y, z) in enumerate(centres):
        o = ((x - 4) % nx, (y - 4) % ny, (z - 4) % nz)
        g = oracle.Geometry(dims, (0, 0, 0), origin=o, wdims=(9, 9, 9))
        xs = [(o[0] + i) % nx for i in range(9)]
        ys = [(o[1] + i) % ny for i in range(9)]
        zs = [(o[2] + i) % nz for i in range(9)]
        win = field_dev[:, zs][:, :, ys][:, :, :, xs].double().cpu().numpy()
        f0 = oracle.init(g, lattice=lattice)
        ref = oracle.run(g, f0, RATES, steps, force_field=win, lattice=lattice)
        assert np.max(np.abs(got[:, k] - ref[:, 4, 4, 4])) < tol, (x, y, z)


def test_largest_fp16_lattice_2_to_30_nodes():
    from paper_1801_04586_amd import Lattice

    dims = (1024, 1024, 1024)
    need = 2 * 27 * (2 ** 30 + 2048) * 2 + 3 * 2 ** 32 + (8 << 30)
    if _free_bytes() < need:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of free device memory")
    gen = torch.Generator(device="cuda").manual_seed(1801)
    field = torch.randn((3, 1024, 1024, 1024), device="cuda", generator=gen, dtype=torch.float32)
    field.mul_(1e-4)
    lat = Lattice(dims, (0, 0, 0), "f16", RATES, force_field=field)
    assert lat.P * 2 * 27 > 2 ** 31  # planes past 2 GiB from the base
    lat.init()
    lat.step(3)
    centres = [(1023, 1023, 1023), (1020, 1023, 1022), (0, 1023, 1023), (517, 3, 1023), (0, 0, 0)]
    _window_check(lat, lat.force_field, dims, "d3q27", 3, centres, 2e-6)
    _, _, tot, nbad = lat.moments(fields=False)
    assert nbad == 0 and abs(tot[0] / 2 ** 30 - 1.0) < 1e-3
    lat.close()
    del lat, field
    torch.cuda.empty_cache()


def test_largest_fp64_lattice_2_to_29_nodes_d3q19():
    from paper_1801_04586_amd import Lattice

    dims = (1024, 1024, 512)
    need = 2 * 19 * (2 ** 29 + 512) * 8 + 3 * 2 ** 32 + (8 << 30)
    if _free_bytes() < need:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of free device memory")
    gen = torch.Generator(device="cuda").manual_seed(1802)
    field = torch.randn((3, 512, 1024, 1024), device="cuda", generator=gen, dtype=torch.float64)
    field.mul_(1e-4)
    lat = Lattice(dims, (0, 0, 0), "f64", RATES, force_field=field, lattice="d3q19")
    lat.init()
    lat.step(2)
    centres = [(1023, 1023, 511), (1000, 1022, 510), (5, 7, 511)]
    _window_check(lat, lat.force_field, dims, "d3q19", 2, centres, 1e-14)
    lat.close()
    del lat, field
    torch.cuda.empty_cache()


def test_empty_calls():
    from paper_1801_04586_amd import Lattice

    dims = (6, 5, 4)
    lat = Lattice(dims, (0, 1, 0), "f32", RATES)
    lat.init()
    before = lat.state.clone()
    lat.step(0)
    assert torch.equal(lat.state, before) and lat.t == 0
    ids = torch.empty(0, dtype=torch.int32, device="cuda")
    out = torch.empty((27, 0), dtype=torch.float64, device="cuda")
    lat.ctx.sample_populations(lat.state, ids, out)
    lat.close()
