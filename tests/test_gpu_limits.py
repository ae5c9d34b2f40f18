"""Edge cases at the limits of the C ABI: the largest lattices the 32-bit plane
offsets allow (N = 2^30 nodes with FP16 storage and an FP32 force field; N =
2^30 with FP32 storage through the fused two-step kernels, periodic and with
walls and solids; N = 2^29 with FP64 storage, D3Q19), checked on sampled nodes
near the last node against the oracle on a window around them; and empty calls
(zero steps, zero samples)."""
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


def _window_check(lat, field_dev, dims, lattice, steps, centres, tol, walls=(0, 0, 0), solid_dev=None):
    """Oracle on a 9^3 window around each centre (wrapped on periodic axes, inside the walls on walled
    ones), started from rest with the window's force field and solid mask; the centre node is exact
    after `steps` <= 4 steps (light cone)."""
    nx, ny, nz = dims
    got = lat.sample(centres)
    for k, (x, y, z) in enumerate(centres):
        o = ((x - 4) % nx, (y - 4) % ny, (z - 4) % nz)
        for a, c, n in zip(range(3), (x, y, z), dims):
            assert not walls[a] or 4 <= c <= n - 5, "window crosses a wall"
        g = oracle.Geometry(dims, walls, origin=o, wdims=(9, 9, 9))
        xs = [(o[0] + i) % nx for i in range(9)]
        ys = [(o[1] + i) % ny for i in range(9)]
        zs = [(o[2] + i) % nz for i in range(9)]
        win = field_dev[:, zs][:, :, ys][:, :, :, xs].double().cpu().numpy()
        sol = None if solid_dev is None else solid_dev[zs][:, ys][:, :, xs].cpu().numpy()
        f0 = oracle.init(g, lattice=lattice)
        ref = oracle.run(g, f0, RATES, steps, force_field=win, lattice=lattice, solid=sol)
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


@pytest.mark.parametrize("walls,frac", [((0, 0, 0), 0.0), ((0, 1, 1), 0.05)], ids=["periodic", "walls_solids"])
def test_largest_fp32_lattice_2_to_30_nodes_fused_pairs(walls, frac):
    from paper_1801_04586_amd import Lattice

    dims = (2048, 1024, 512)
    N = 2 ** 30
    need = 2 * 27 * (N + 1024) * 4 + 3 * N * 4 + 5 * N + N // 4 + (8 << 30)
    if _free_bytes() < need:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of free device memory")
    gen = torch.Generator(device="cuda").manual_seed(1803)
    field = torch.randn((3, 512, 1024, 2048), device="cuda", generator=gen, dtype=torch.float32)
    field.mul_(1e-4)
    if walls == (0, 0, 0):
        centres = [(2047, 1023, 511), (0, 0, 0), (1024, 1023, 0), (31, 11, 255)]
    else:
        centres = [(2047, 1019, 507), (0, 4, 4), (1234, 511, 255), (2016, 1019, 4)]
    solid = None
    if frac:
        solid = (torch.rand((512, 1024, 2048), device="cuda", generator=gen) < frac).to(torch.uint8)
        for x, y, z in centres:
            solid[z, y, x] = 0
    lat = Lattice(dims, walls, "f32", RATES, force_field=field, solid=solid)
    assert lat.uses_fused_pairs
    assert lat.P * 4 * 27 > 2 ** 32  # planes past 4 GiB from the base
    lat.init()
    lat.step(4)
    _window_check(lat, lat.force_field, dims, "d3q27", 4, centres, 1e-7, walls, solid)
    _, _, tot, nbad = lat.moments(fields=False)
    fluid = N if solid is None else int(N - solid.sum(dtype=torch.int64).item())
    assert nbad == 0 and abs(tot[0] / fluid - 1.0) < 1e-6
    lat.close()
    del lat, field, solid
    torch.cuda.empty_cache()


@pytest.mark.parametrize("fused", [True, False], ids=["fused_pairs", "single_steps"])
def test_largest_fp64_lattice_2_to_29_nodes_d3q19(fused):
    """The largest FP64 lattice (2^29 nodes, D3Q19, periodic): the fused pair it takes by default, and
    single steps, against the oracle on windows around nodes at the ends of the 32-bit byte offsets."""
    from paper_1801_04586_amd import Lattice

    dims = (1024, 1024, 512)
    need = 2 * 19 * (2 ** 29 + 512) * 8 + 3 * 2 ** 32 + (8 << 30)
    if _free_bytes() < need:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of free device memory")
    gen = torch.Generator(device="cuda").manual_seed(1802)
    field = torch.randn((3, 512, 1024, 1024), device="cuda", generator=gen, dtype=torch.float64)
    field.mul_(1e-4)
    lat = Lattice(dims, (0, 0, 0), "f64", RATES, force_field=field, lattice="d3q19")
    assert lat.uses_fused_pairs
    lat.set_fused_steps(fused)
    assert lat.uses_fused_pairs == fused
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
