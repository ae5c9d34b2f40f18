"""clbm_adjoint_step_noalloc (the adjoint step for callers that cannot allocate) against
clbm_adjoint_step, through the C ABI: two calls in a row, the second on a smaller lattice, give
bitwise the same lambda, dJ/dF and dJ/ds; lattices above its limit are refused before any work."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

RATES = np.array([1.0, 1.0, 1.55, 1.2, 1.3, 0.9, 1.1, 1.25, 0.95, 1.05])


def _adjoint_pair(dims, walls, solid_frac, storage, seed):
    from paper_1801_04586_amd import Lattice

    g = oracle.Geometry(dims, walls)
    rho0, u0 = workloads.random_state_fields(dims, seed, du=0.04, drho=0.01)
    f0 = oracle.init(g, rho0, u0) + workloads.random_populations_perturbation(dims, seed + 1, 5e-4)
    solid = workloads.random_solids(dims, solid_frac, seed + 3) if solid_frac else None
    field = workloads.gaussian_force(dims, 1e-4, seed + 2)
    lat = Lattice(dims, walls, storage, RATES, force=(1e-5, -2e-5, 5e-6), force_field=field, solid=solid)
    lat.set_populations(torch.from_numpy(f0))
    real = lat.real
    ln = torch.from_numpy(np.random.default_rng(seed + 4).normal(0, 1, (27,) + g.shape)).to("cuda", real)
    ln = ln.contiguous()
    outs = []
    for noalloc in (False, True):
        lo = torch.empty_like(ln)
        gF = torch.full((3,) + g.shape, 0.25, dtype=real, device="cuda")
        gs = torch.full((10,), 0.5, dtype=torch.float64, device="cuda")
        step = lat.ctx.adjoint_step_noalloc if noalloc else lat.ctx.adjoint_step
        step(lat.state, ln, lo, gF, gs)
        torch.cuda.synchronize()
        outs.append((lo, gF, gs))
    lat.close()
    return outs


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_noalloc_adjoint_step_equals_the_allocating_one_on_two_calls_in_a_row(storage):
    # first call: 552 960 nodes, 2160 blocks of partial sums, so the fold into the scratch's second
    # part runs too; second call: a smaller lattice, whose results must not see the first one's
    for dims, walls, solid_frac, seed in (((96, 80, 72), (0, 1, 1), 0.1, 11), ((7, 6, 5), (1, 1, 1), 0.2, 12)):
        (lo_a, gF_a, gs_a), (lo_b, gF_b, gs_b) = _adjoint_pair(dims, walls, solid_frac, storage, seed)
        assert torch.equal(lo_a, lo_b), dims
        assert torch.equal(gF_a, gF_b), dims
        assert torch.equal(gs_a, gs_b), dims
        assert gs_b[0].item() == 0.5 and gs_b[1].item() == 0.5 and (gs_b[2:] != 0.5).any()


def test_noalloc_adjoint_step_refuses_lattices_above_its_limit():
    from paper_1801_04586_amd import ClbmError, Lattice, load_library

    lib = load_library()
    assert lib.clbm_adjoint_noalloc_max_nodes() == 2 ** 25
    dims = (256, 256, 513)  # 2^25 + 65536 nodes
    lat = Lattice(dims, (0, 0, 0), "f32", RATES, plane_stride=0)
    n = int(np.prod(dims))
    lam = torch.zeros((27, n), dtype=torch.float32, device="cuda")
    lam2 = torch.zeros_like(lam)
    with pytest.raises(ClbmError) as e:
        lat.ctx.adjoint_step_noalloc(lat.state, lam, lam2)
    assert e.value.code == 1 and "2^25" in str(e.value)
    torch.cuda.synchronize()
    lat.close()
