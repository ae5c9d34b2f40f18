"""Parity of the HIP path (through the C ABI) against the FP64 CPU oracle.

Every case starts both sides from the same seeded inputs (workloads/) and
compares pre-collision populations or macroscopic fields element by element.
Tolerances:
  * FP64 storage: 1e-13 absolute on populations (O(1) values, rounding order
    of the factorised transforms differs from the dense oracle);
  * FP32 deviation storage: bounded by FP32 rounding of deviations and FP32
    arithmetic on O(1e-2) moments, 5e-8 absolute;
  * FP16 / BF16 storage: one storage rounding per step of deviations
    (2^-11 / 2^-8 relative) -- checked against the oracle after one step.
"""
from __future__ import annotations

import itertools

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

RATES = np.array([1.0, 1.0, 1.6, 1.2, 1.3, 0.9, 1.1, 1.25, 0.95, 1.05])
# every rate above second order equal to one (the setting of Sec. III): the kernels
# take a separate collision path for it
RATES_H1 = np.array([1.0, 1.0, 1.6, 1.2, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0])
TOL = {"f64": 1e-13, "f32": 5e-8, "f16": 1e-5, "bf16": 8e-5}


def _lattice(dims, walls, storage, rates=RATES, force=(0.0, 0.0, 0.0), field=None, solid=None):
    from paper_1801_04586_amd import Lattice

    return Lattice(dims, walls, storage, rates, force=force, force_field=field, solid=solid)


def _random_start(dims, walls, seed, solid=None):
    g = oracle.Geometry(dims, walls)
    rho0, u0 = workloads.random_state_fields(dims, seed, du=0.05, drho=0.02)
    f0 = oracle.init(g, rho0, u0) + workloads.random_populations_perturbation(dims, seed + 1, 1e-3)
    return g, f0


def _fluid(solid, shape):
    return np.ones(shape, bool) if solid is None else (solid == 0)


def _compare(dims, walls, storage, steps, seed, with_field=True, solid_frac=0.0, force=(2e-5, -1e-5, 3e-6),
             rates=RATES):
    solid = workloads.random_solids(dims, solid_frac, seed + 5) if solid_frac else None
    g, f0 = _random_start(dims, walls, seed, solid)
    field = workloads.gaussian_force(dims, 1e-4, seed + 2) if with_field else None
    lat = _lattice(dims, walls, storage, rates=rates, force=force, field=field, solid=solid)
    lat.set_populations(torch.from_numpy(f0))
    start = lat.populations().cpu().numpy()  # f0 rounded to the storage type
    fl = _fluid(solid, g.shape)
    if storage == "f64":
        assert np.array_equal(start[:, fl], f0[:, fl])
    ref = oracle.run(g, start, rates, steps, force=force, force_field=field, solid=solid)
    lat.step(steps)
    got = lat.populations().cpu().numpy()
    lat.close()
    return np.max(np.abs(got[:, fl] - ref[:, fl]))


# ----------------------------------------------------------------------------- initial state and round trips
def test_init_is_the_generalized_equilibrium():
    dims, walls = (9, 8, 7), (0, 1, 1)
    rho0, u0 = workloads.random_state_fields(dims, 3)
    g = oracle.Geometry(dims, walls)
    ref = oracle.init(g, rho0, u0)
    for storage, tol in (("f64", 1e-15), ("f32", 1e-9)):
        lat = _lattice(dims, walls, storage)
        lat.init(rho0, u0)
        got = lat.populations().cpu().numpy()
        assert np.max(np.abs(got - ref)) < tol, storage
        lat.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16"])
def test_set_get_populations_roundtrip(storage):
    dims, walls = (11, 5, 6), (1, 0, 1)
    solid = workloads.random_solids(dims, 0.2, 4)
    g, f0 = _random_start(dims, walls, 5)
    lat = _lattice(dims, walls, storage, solid=solid)
    lat.set_populations(torch.from_numpy(f0))
    got = lat.populations().cpu().numpy()
    fl = solid == 0
    w = oracle.equilibrium(1.0, [0, 0, 0])[:, None]
    err = np.abs(got[:, fl] - f0[:, fl]) / np.maximum(np.abs(f0[:, fl] - w), 1e-30)
    rel = {"f64": 0.0, "f32": 2.0 ** -24, "f16": 2.0 ** -11, "bf16": 2.0 ** -8}[storage]
    if storage == "f64":
        assert np.array_equal(got[:, fl], f0[:, fl])
    else:
        # one round-to-nearest of the deviation f - w (FP16 subnormals: absolute 2^-25)
        assert np.all((err <= rel * 1.0001) | (np.abs(got[:, fl] - f0[:, fl]) <= 2.0 ** -25))
    assert np.all(got[:, ~fl] == 0.0)
    lat.close()


# ----------------------------------------------------------------------------- one and several steps
WALL_COMBOS = list(itertools.product((0, 1), repeat=3))


@pytest.mark.parametrize("walls", WALL_COMBOS)
def test_step_parity_f64_every_wall_combination(walls):
    dims = (5, 7, 3)
    assert _compare(dims, walls, "f64", 1, 11) < TOL["f64"]
    assert _compare(dims, walls, "f64", 10, 12, solid_frac=0.15) < TOL["f64"]


@pytest.mark.parametrize("dims", [(1, 1, 9), (2, 3, 5), (67, 3, 2), (16, 1, 1), (3, 70, 3), (1, 33, 17)])
def test_step_parity_f64_odd_and_degenerate_shapes(dims):
    assert _compare(dims, (0, 0, 0), "f64", 4, 21) < TOL["f64"]
    assert _compare(dims, (1, 1, 1), "f64", 4, 22) < TOL["f64"]


def test_step_parity_f64_several_blocks_and_ragged_tail():
    # 23 * 19 * 13 = 5681 nodes: 22 full blocks of 256 and a ragged tail
    assert _compare((23, 19, 13), (0, 1, 0), "f64", 6, 31, solid_frac=0.1) < TOL["f64"]
    assert _compare((23, 19, 13), (0, 0, 0), "f64", 6, 32, with_field=False) < TOL["f64"]


@pytest.mark.parametrize("dims,walls", [((316, 312, 17), (0, 1, 1)), ((400, 250, 12), (1, 0, 0))])
def test_step_parity_f64_solids_on_large_planes(dims, walls):
    """With solids and at least 98 304 nodes per plane the step kernel visits nodes in groups of eight
    z planes: two whole groups and a partial one, or one and a partial one."""
    assert _compare(dims, walls, "f64", 2, 51, solid_frac=0.2) < TOL["f64"]


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("walls,solid_frac", [((0, 0, 0), 0.0), ((0, 1, 1), 0.0), ((1, 0, 1), 0.2)])
def test_step_parity_reduced_storage_one_step(storage, walls, solid_frac):
    assert _compare((13, 9, 7), walls, storage, 1, 41, solid_frac=solid_frac) < TOL[storage]


def test_step_parity_f32_ten_steps():
    assert _compare((13, 9, 7), (0, 1, 0), "f32", 10, 43, solid_frac=0.1) < 2e-7


@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16"])
@pytest.mark.parametrize("walls,solid_frac,with_field", [((0, 0, 0), 0.0, True), ((0, 1, 1), 0.0, False),
                                                         ((1, 0, 1), 0.2, True)])
def test_step_parity_high_order_rates_one(storage, walls, solid_frac, with_field):
    steps = 5 if storage in ("f64", "f32") else 1
    tol = {"f64": 1e-13, "f32": 1.5e-7}.get(storage, TOL[storage])
    err = _compare((23, 19, 13), walls, storage, steps, 61, with_field=with_field, solid_frac=solid_frac,
                   rates=RATES_H1)
    assert err < tol, err


def test_high_order_rates_one_path_agrees_with_general_path():
    """Rates one ulp above one take the general collision; the results may differ
    only by rounding (FP64)."""
    dims, walls = (17, 11, 9), (0, 1, 0)
    g, f0 = _random_start(dims, walls, 71)
    near = RATES_H1.copy()
    near[4:] = np.nextafter(1.0, 2.0)
    out = []
    for r in (RATES_H1, near):
        lat = _lattice(dims, walls, "f64", rates=r, force=(1e-5, 0, 0))
        lat.set_populations(torch.from_numpy(f0))
        lat.step(8)
        out.append(lat.populations().cpu().numpy())
        lat.close()
    assert np.max(np.abs(out[0] - out[1])) < 1e-13


# ----------------------------------------------------------------------------- moments and conservation
def test_moments_match_oracle_and_totals():
    dims, walls = (10, 9, 8), (0, 1, 0)
    solid = workloads.random_solids(dims, 0.1, 51)
    g, f0 = _random_start(dims, walls, 52)
    field = workloads.gaussian_force(dims, 1e-4, 53)
    force = (1e-5, 0.0, -2e-5)
    lat = _lattice(dims, walls, "f64", force=force, field=field, solid=solid)
    lat.set_populations(torch.from_numpy(f0))
    rho, u, totals, nbad = lat.moments()
    rr, ur = oracle.macro(g, f0, force=force, force_field=field, solid=solid)
    fl = solid == 0
    assert nbad == 0
    assert np.max(np.abs(rho.cpu().numpy()[fl] - rr[fl])) < 1e-14
    assert np.max(np.abs(u.cpu().numpy()[:, fl] - ur[:, fl])) < 1e-14
    assert abs(totals[0] - rr[fl].sum()) < 1e-12
    assert np.max(np.abs(totals[1:] - (rr[None] * ur)[:, fl].sum(axis=1))) < 1e-12
    lat.close()


@pytest.mark.parametrize("storage,rel", [("f64", 1e-13), ("f32", 1e-9)])
def test_global_mass_conserved_with_walls_and_solids(storage, rel):
    dims, walls = (24, 20, 16), (0, 1, 1)
    solid = workloads.random_solids(dims, 0.2, 61)
    g, f0 = _random_start(dims, walls, 62)
    lat = _lattice(dims, walls, storage, force=(1e-5, 0, 0), solid=solid)
    lat.set_populations(torch.from_numpy(f0))
    m0 = lat.moments(fields=False)[2][0]
    lat.step(200)
    m1 = lat.moments(fields=False)[2][0]
    assert abs(m1 - m0) <= rel * m0
    lat.close()


def test_periodic_momentum_grows_by_total_force():
    dims = (12, 10, 8)
    g, f0 = _random_start(dims, (0, 0, 0), 71)
    field = workloads.gaussian_force(dims, 1e-5, 72)
    lat = _lattice(dims, (0, 0, 0), "f64", force=(1e-6, 2e-6, 0.0), field=field)
    lat.set_populations(torch.from_numpy(f0))
    p0 = lat.moments(fields=False)[2][1:]
    lat.step(50)
    p1 = lat.moments(fields=False)[2][1:]
    n = np.prod(dims)
    expect = 50 * (field.reshape(3, -1).sum(axis=1) + n * np.array([1e-6, 2e-6, 0.0]))
    assert np.max(np.abs(p1 - p0 - expect)) < 1e-12
    lat.close()


def test_nonfinite_state_is_reported():
    dims = (4, 4, 4)
    g, f0 = _random_start(dims, (0, 0, 0), 81)
    f0[3, 1, 2, 3] = np.nan
    lat = _lattice(dims, (0, 0, 0), "f32")
    lat.set_populations(torch.from_numpy(f0))
    _, _, _, nbad = lat.moments(fields=False)
    assert nbad >= 1
    lat.close()


# ----------------------------------------------------------------------------- write coverage and determinism
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_every_fluid_entry_is_written(storage):
    dims, walls = (19, 11, 6), (1, 1, 0)
    solid = workloads.random_solids(dims, 0.25, 91)
    g, f0 = _random_start(dims, walls, 92)
    lat = _lattice(dims, walls, storage, solid=solid)
    lat.set_populations(torch.from_numpy(f0))
    lat.other.fill_(float("nan"))
    lat.step(1)
    st = lat.view().to(torch.float64).cpu().numpy()
    assert not np.isnan(st[:, solid == 0]).any()
    lat.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_plane_stride_changes_nothing_but_the_layout(storage):
    """The default padded plane stride and a dense one (P = N) give identical results, and the
    padding is never written."""
    from paper_1801_04586_amd import Lattice

    dims, walls = (21, 13, 7), (0, 1, 1)
    solid = workloads.random_solids(dims, 0.1, 111)
    g, f0 = _random_start(dims, walls, 112)
    field = workloads.gaussian_force(dims, 1e-4, 113)
    out = []
    for ps in (None, 0):
        lat = Lattice(dims, walls, storage, RATES, force=(1e-5, 0, 0), force_field=field, solid=solid,
                      plane_stride=ps)
        assert (lat.P > lat.n) == (ps is None)
        lat.set_populations(torch.from_numpy(f0))
        lat.step(7)
        out.append(lat.populations().cpu().numpy())
        for b in lat.bufs:
            assert torch.count_nonzero(b[:, lat.n:]).item() == 0
        lat.close()
    assert np.array_equal(out[0], out[1])


def test_runs_are_bitwise_deterministic():
    dims, walls = (33, 17, 9), (0, 1, 0)
    g, f0 = _random_start(dims, walls, 101)
    outs = []
    for _ in range(2):
        lat = _lattice(dims, walls, "f32", force=(1e-5, 0, 0))
        lat.set_populations(torch.from_numpy(f0))
        lat.step(25)
        outs.append(lat.state.clone())
        lat.close()
    assert torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_step_parity_with_a_force_scale_and_fused_pairs(storage):
    """clbm_set_force with a scale other than 1 (time-dependent forcing): the kernels use
    F = uniform + scale * field; the oracle is given the scaled field.  Both storage types run fused
    pairs (the link-table variant: the duct has walls)."""
    dims, walls = (37, 13, 16), (0, 1, 0)
    g, f0 = _random_start(dims, walls, 91)
    field = workloads.gaussian_force(dims, 1e-4, 92)
    force, scale = (2e-5, -1e-5, 3e-6), -3.25
    lat = _lattice(dims, walls, storage, force=force, field=field)
    lat.set_force(force, field, scale)
    lat.set_fused_steps(True)
    assert lat.uses_fused_pairs
    lat.set_populations(torch.from_numpy(f0))
    start = lat.populations().cpu().numpy()
    Fs = scale * lat.force_field.double().cpu().numpy()
    ref = oracle.run(g, start, RATES, 4, force=force, force_field=Fs)
    lat.step(4)
    err = np.max(np.abs(lat.populations().cpu().numpy() - ref))
    lat.close()
    assert err < (TOL["f64"] if storage == "f64" else 2e-7), err
