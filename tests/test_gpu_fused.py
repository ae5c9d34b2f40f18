"""Fused two-step launches (clbm_run on FP32 periodic lattices without solids)
are bitwise identical to single steps, across ragged tiles, thin lattices, odd
step counts, both collision paths and with or without a force field; and they
match the oracle."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

RATES = np.array([1.0, 1.0, 1.6, 1.2, 1.3, 0.9, 1.1, 1.25, 0.95, 1.05])
RATES_H1 = np.array([1.0, 1.0, 1.6, 1.2, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0])  # rates above second order = 1


def _start(dims, seed):
    g = oracle.Geometry(dims)
    rho0, u0 = workloads.random_state_fields(dims, seed, du=0.05, drho=0.02)
    return g, oracle.init(g, rho0, u0) + workloads.random_populations_perturbation(dims, seed + 1, 1e-3)


def _run(dims, storage, steps, fused, f0, field, rates=RATES):
    from paper_1801_04586_amd import Lattice

    lat = Lattice(dims, (0, 0, 0), storage, rates, force=(1e-5, -3e-6, 2e-6), force_field=field)
    lat.set_fused_steps(fused)
    lat.set_populations(torch.from_numpy(f0))
    lat.step(steps)
    out = lat.state.clone()
    pops = lat.populations().cpu().numpy()
    lat.close()
    return out, pops


@pytest.mark.parametrize("dims", [(67, 19, 13), (32, 8, 16), (16, 8, 3), (5, 7, 2), (1, 1, 9), (33, 9, 40),
                                  (96, 17, 1)])
@pytest.mark.parametrize("storage", ["f32"])
@pytest.mark.parametrize("rates", [RATES, RATES_H1], ids=["general", "high1"])
def test_fused_pairs_are_bitwise_single_steps(dims, storage, rates):
    g, f0 = _start(dims, 3)
    field = workloads.gaussian_force(dims, 1e-4, 4)
    for steps in (2, 5):
        a, _ = _run(dims, storage, steps, True, f0, field, rates)
        b, _ = _run(dims, storage, steps, False, f0, field, rates)
        assert torch.equal(a, b), (dims, storage, steps)


@pytest.mark.parametrize("rates", [RATES, RATES_H1], ids=["general", "high1"])
def test_fused_pairs_without_force_field(rates):
    dims = (40, 24, 10)
    g, f0 = _start(dims, 5)
    a, _ = _run(dims, "f32", 6, True, f0, None, rates)
    b, _ = _run(dims, "f32", 6, False, f0, None, rates)
    assert torch.equal(a, b)


def test_fused_pairs_apply_to_fp32_periodic_lattices_only():
    from paper_1801_04586_amd import Lattice

    dims = (8, 8, 8)
    cases = [("f32", (0, 0, 0), None, True), ("f64", (0, 0, 0), None, False), ("f16", (0, 0, 0), None, False),
             ("bf16", (0, 0, 0), None, False), ("f32", (0, 1, 0), None, False),
             ("f32", (0, 0, 0), workloads.random_solids(dims, 0.1, 9), False)]
    for storage, walls, solid, fused in cases:
        lat = Lattice(dims, walls, storage, RATES, solid=solid)
        assert lat.uses_fused_pairs == fused, (storage, walls)
        lat.close()


def test_fused_run_matches_oracle():
    dims = (37, 11, 6)
    g, f0 = _start(dims, 7)
    field = workloads.gaussian_force(dims, 1e-4, 8)
    from paper_1801_04586_amd import Lattice

    lat = Lattice(dims, (0, 0, 0), "f32", RATES, force=(1e-5, -3e-6, 2e-6), force_field=field)
    lat.set_populations(torch.from_numpy(f0))
    start = lat.populations().cpu().numpy()
    lat.step(4)
    got = lat.populations().cpu().numpy()
    ref = oracle.run(g, start, RATES, 4, force=(1e-5, -3e-6, 2e-6), force_field=lat.force_field.double().cpu().numpy())
    assert np.max(np.abs(got - ref)) < 1e-7
    lat.close()
