"""The step path records into a HIP graph (torch.cuda.CUDAGraph on ROCm): clbm_run
launches kernels only, with no allocation, copy or memset, so a captured run of
fused step pairs replays as the eager run does.  Each replay is checked bitwise
against eager steps, with the program's own eager work and synchronisations
between the replays."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

RATES = np.array([1.0, 1.0, 1.6, 1.2, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0])


def _lattice(dims, walls, solid, field, storage):
    from paper_1801_04586_amd import Lattice

    lat = Lattice(dims, walls, storage, RATES, force=(1e-5, 0.0, 0.0), force_field=field, solid=solid)
    lat.set_fused_steps(True)
    return lat


@pytest.mark.parametrize("storage", ["f32", "f64"])
@pytest.mark.parametrize("walls,frac", [((0, 0, 0), 0.0), ((0, 1, 1), 0.1)], ids=["periodic", "walls_solids"])
def test_captured_run_replays_bitwise_like_eager_steps(walls, frac, storage):
    dims = (70, 30, 24)
    g = oracle.Geometry(dims, walls)
    rho0, u0 = workloads.random_state_fields(dims, 91, du=0.05, drho=0.02)
    f0 = oracle.init(g, rho0, u0) + workloads.random_populations_perturbation(dims, 92, 1e-3)
    field = workloads.gaussian_force(dims, 1e-4, 93)
    solid = workloads.random_solids(dims, frac, 94) if frac else None

    # eager reference: three rounds of 8 steps (four fused launches each)
    ref = _lattice(dims, walls, solid, field, storage)
    assert ref.uses_fused_pairs
    ref.set_populations(torch.from_numpy(f0))
    expected = []
    for _ in range(3):
        ref.step(8)
        expected.append(ref.state.clone())
    ref.close()

    lat = _lattice(dims, walls, solid, field, storage)
    lat.set_populations(torch.from_numpy(f0))
    start = lat.state.clone()
    lat.step(2)  # first launches outside the capture (the context sizes its fused launches once)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            lat.step(8)  # an even number of launches: the state ends in the buffer it started in
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    lat.state.copy_(start)
    lat.t = 0
    torch.cuda.synchronize()
    for r in range(3):
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(lat.state, expected[r]), r
        _, _, tot, nbad = lat.moments(fields=False)  # eager work between replays
        assert nbad == 0 and np.isfinite(tot[0])
    lat.close()
