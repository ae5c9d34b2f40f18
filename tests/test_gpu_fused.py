"""Fused two-step launches (clbm_run on FP32 and FP64 D3Q27 lattices with the cascaded or the
MRT collision, and on FP32 and FP64 D3Q19 lattices: periodic, walled, moving walls, solid nodes) are
bitwise identical to single steps,
across ragged tiles, thin lattices, odd step counts, both collision paths, with
or without a force field, every wall combination, random solids and packed
spheres; and they match the oracle."""
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
@pytest.mark.parametrize("storage", ["f32", "f64"])
@pytest.mark.parametrize("rates", [RATES, RATES_H1], ids=["general", "high1"])
def test_fused_pairs_are_bitwise_single_steps(dims, storage, rates):
    g, f0 = _start(dims, 3)
    field = workloads.gaussian_force(dims, 1e-4, 4)
    for steps in (2, 5):
        a, _ = _run(dims, storage, steps, True, f0, field, rates)
        b, _ = _run(dims, storage, steps, False, f0, field, rates)
        assert torch.equal(a, b), (dims, storage, steps)


@pytest.mark.parametrize("storage", ["f32", "f64"])
@pytest.mark.parametrize("rates", [RATES, RATES_H1], ids=["general", "high1"])
def test_fused_pairs_without_force_field(storage, rates):
    dims = (40, 24, 10)
    g, f0 = _start(dims, 5)
    a, _ = _run(dims, storage, 6, True, f0, None, rates)
    b, _ = _run(dims, storage, 6, False, f0, None, rates)
    assert torch.equal(a, b)


def test_fused_pairs_apply_to_fp32_and_fp64_lattices():
    from paper_1801_04586_amd import Lattice

    dims = (8, 8, 8)
    sol = workloads.random_solids(dims, 0.1, 9)
    lid = {(1, 1): (0.01, 0.0, 0.0)}
    cases = [("f32", (0, 0, 0), None, None, "d3q27", "cascaded", True),
             ("f64", (0, 0, 0), None, None, "d3q27", "cascaded", True),
             ("f16", (0, 0, 0), None, None, "d3q27", "cascaded", False),
             ("bf16", (0, 0, 0), None, None, "d3q27", "cascaded", False),
             ("f32", (0, 1, 0), None, None, "d3q27", "cascaded", True),
             ("f32", (0, 0, 0), sol, None, "d3q27", "cascaded", True),
             ("f32", (1, 1, 1), sol, None, "d3q27", "cascaded", True),
             ("f64", (0, 1, 0), sol, None, "d3q27", "cascaded", True),
             ("f32", (0, 1, 0), sol, lid, "d3q27", "cascaded", True),
             ("f32", (1, 1, 1), None, lid, "d3q27", "cascaded", True),
             ("f32", (0, 1, 0), None, None, "d3q19", "cascaded", True),
             ("f32", (1, 1, 1), sol, lid, "d3q19", "cascaded", True),
             ("f64", (0, 1, 0), None, None, "d3q19", "cascaded", True),
             ("f64", (0, 0, 0), None, None, "d3q19", "cascaded", True),
             ("f64", (0, 0, 0), sol, None, "d3q27", "cascaded", True),
             ("f64", (1, 1, 1), sol, lid, "d3q19", "cascaded", True),
             ("f32", (0, 1, 0), None, None, "d3q27", "mrt", True),
             ("f32", (1, 1, 1), sol, lid, "d3q27", "mrt", True),
             ("f64", (0, 1, 0), None, None, "d3q27", "mrt", True),
             ("f64", (0, 0, 0), None, None, "d3q27", "mrt", True)]
    for storage, walls, solid, wv, lattice, coll, fused in cases:
        lat = Lattice(dims, walls, storage, RATES, solid=solid, wall_velocity=wv, lattice=lattice, collision=coll)
        assert not lat.uses_fused_pairs  # 8^3 is too small to fill the device: single steps by default
        lat.set_fused_steps(True)
        assert lat.uses_fused_pairs == fused, (storage, walls, solid is not None, wv, lattice, coll)
        lat.set_fused_steps(False)
        assert not lat.uses_fused_pairs
        lat.close()


def test_fused_option_flags():
    from paper_1801_04586_amd import Lattice
    from paper_1801_04586_amd.clbm import ClbmError

    lat = Lattice((8, 8, 8), (0, 0, 0), "f32", RATES)
    for opts, fused in ((0, False), (1, False), (2, True)):
        lat.ctx.set_options(opts)
        assert lat.uses_fused_pairs == fused, opts
    for bad in (3, 4, 0x80000000):
        with pytest.raises(ClbmError) as e:
            lat.ctx.set_options(bad)
        assert e.value.code == 1
    assert lat.uses_fused_pairs  # a refused call leaves the options as they were
    lat.close()


def test_fused_pairs_by_default_only_on_lattices_that_fill_the_device():
    """Default rule: tile columns (32 x 12; 32 x 16 for FP64 with the cascaded collision) times z chunks
    of 8 planes must give two blocks per compute unit."""
    from paper_1801_04586_amd import Lattice

    cus = torch.cuda.get_device_properties(0).multi_processor_count
    for dims, walls, storage, coll in (((64, 64, 64), (0, 1, 0), "f32", "cascaded"),
                                       ((128, 128, 128), (0, 0, 0), "f32", "cascaded"),
                                       ((256, 96, 64), (1, 1, 1), "f32", "cascaded"),
                                       ((128, 128, 128), (0, 0, 0), "f64", "cascaded"),
                                       ((128, 112, 128), (0, 0, 0), "f64", "cascaded"),
                                       ((128, 112, 128), (0, 0, 0), "f64", "mrt"),
                                       ((96, 96, 64), (0, 0, 0), "f64", "cascaded")):
        rows = 16 if storage == "f64" and coll == "cascaded" else 12
        blocks = -(-dims[0] // 32) * -(-dims[1] // rows) * max(dims[2] // 8, 1)
        lat = Lattice(dims, walls, storage, RATES, collision=coll)
        assert lat.uses_fused_pairs == (blocks >= 2 * cus), (dims, storage, coll, blocks, cus)
        lat.close()


def _run_solid(dims, walls, solid, steps, fused, f0, field, rates=RATES, wall_velocity=None, collision="cascaded",
               storage="f32"):
    from paper_1801_04586_amd import Lattice

    lat = Lattice(dims, walls, storage, rates, force=(1e-5, -3e-6, 2e-6), force_field=field, solid=solid,
                  wall_velocity=wall_velocity, collision=collision)
    lat.set_fused_steps(fused)
    assert lat.uses_fused_pairs == fused
    lat.set_populations(torch.from_numpy(f0))
    lat.step(steps)
    out = lat.state.clone()
    pops = lat.populations().cpu().numpy()
    lat.close()
    return out, pops


def _start_walls(dims, walls, seed):
    g = oracle.Geometry(dims, walls)
    rho0, u0 = workloads.random_state_fields(dims, seed, du=0.05, drho=0.02)
    return g, oracle.init(g, rho0, u0) + workloads.random_populations_perturbation(dims, seed + 1, 1e-3)


@pytest.mark.parametrize("dims,walls", [((67, 19, 13), (0, 1, 1)), ((32, 24, 16), (0, 0, 0)), ((33, 9, 40), (1, 1, 1)),
                                        ((5, 7, 2), (1, 0, 1)), ((96, 17, 1), (0, 1, 0)), ((1, 13, 9), (0, 1, 1)),
                                        ((40, 12, 3), (0, 0, 1))])
@pytest.mark.parametrize("rates", [RATES, RATES_H1], ids=["general", "high1"])
@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_fused_pairs_with_solids_are_bitwise_single_steps(dims, walls, rates, storage):
    g, f0 = _start_walls(dims, walls, 21)
    field = workloads.gaussian_force(dims, 1e-4, 22)
    solid = workloads.random_solids(dims, 0.2, 23)
    for steps in (2, 5):
        a, _ = _run_solid(dims, walls, solid, steps, True, f0, field, rates, storage=storage)
        b, _ = _run_solid(dims, walls, solid, steps, False, f0, field, rates, storage=storage)
        assert torch.equal(a, b), (dims, walls, steps, storage)


def test_fused_pairs_with_packed_spheres_and_without_force_field():
    dims, walls = (70, 40, 36), (0, 1, 1)
    g, f0 = _start_walls(dims, walls, 31)
    solid, _, _ = workloads.porous_spheres(dims, walls, 3.0, 6.0, 0.2, 32)
    a, _ = _run_solid(dims, walls, solid, 6, True, f0, None, RATES_H1)
    b, _ = _run_solid(dims, walls, solid, 6, False, f0, None, RATES_H1)
    assert torch.equal(a, b)


def test_fused_pairs_with_walls_and_an_all_fluid_mask():
    """A solid mask without solid nodes still gives the lattice a link table: walls alone then take the
    fused path's bounce-back."""
    dims, walls = (34, 26, 11), (1, 1, 0)
    g, f0 = _start_walls(dims, walls, 41)
    solid = np.zeros((11, 26, 34), np.uint8)
    a, _ = _run_solid(dims, walls, solid, 4, True, f0, None)
    b, _ = _run_solid(dims, walls, solid, 4, False, f0, None)
    assert torch.equal(a, b)


@pytest.mark.parametrize("dims,walls", [((67, 19, 13), (0, 1, 0)), ((33, 9, 40), (1, 1, 1)), ((5, 7, 2), (1, 0, 1)),
                                        ((40, 12, 3), (0, 0, 1)), ((1, 13, 9), (0, 1, 1))])
@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_fused_pairs_with_walls_only_are_bitwise_single_steps(dims, walls, storage):
    g, f0 = _start_walls(dims, walls, 61)
    field = workloads.gaussian_force(dims, 1e-4, 62)
    for steps in (2, 5):
        a, _ = _run_solid(dims, walls, None, steps, True, f0, field, storage=storage)
        b, _ = _run_solid(dims, walls, None, steps, False, f0, field, storage=storage)
        assert torch.equal(a, b), (dims, walls, steps, storage)


def _moving_faces(walls, seed):
    rng = np.random.default_rng(seed)
    return {(a, sd): tuple(0.05 * rng.standard_normal(3)) for a in range(3) if walls[a] for sd in (0, 1)}


@pytest.mark.parametrize("dims,walls,frac", [((38, 14, 9), (0, 1, 0), 0.0), ((35, 13, 11), (1, 1, 1), 0.0),
                                             ((35, 13, 11), (1, 1, 1), 0.15), ((20, 30, 7), (0, 1, 1), 0.1)])
@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_fused_pairs_with_moving_walls_are_bitwise_single_steps(dims, walls, frac, storage):
    """Every face of every walled axis moves, so edge and corner links cross two or three moving faces."""
    g, f0 = _start_walls(dims, walls, 71)
    solid = workloads.random_solids(dims, frac, 72) if frac else None
    wv = _moving_faces(walls, 73)
    for steps in (2, 3):
        a, _ = _run_solid(dims, walls, solid, steps, True, f0, None, RATES_H1, wv, storage=storage)
        b, _ = _run_solid(dims, walls, solid, steps, False, f0, None, RATES_H1, wv, storage=storage)
        assert torch.equal(a, b), (dims, walls, frac, steps, storage)


@pytest.mark.parametrize("storage,tol", [("f32", 1e-7), ("f64", 1e-14)])
def test_fused_run_with_moving_walls_matches_oracle(storage, tol):
    dims, walls = (36, 15, 8), (1, 1, 1)
    g, f0 = _start_walls(dims, walls, 81)
    wv = _moving_faces(walls, 82)
    from paper_1801_04586_amd import Lattice

    lat = Lattice(dims, walls, storage, RATES, force=(1e-5, -3e-6, 2e-6), wall_velocity=wv)
    lat.set_fused_steps(True)
    assert lat.uses_fused_pairs
    lat.set_populations(torch.from_numpy(f0))
    start = lat.populations().cpu().numpy()
    lat.step(4)
    got = lat.populations().cpu().numpy()
    ref = oracle.run(g, start, RATES, 4, force=(1e-5, -3e-6, 2e-6), wall_velocity=wv)
    assert np.max(np.abs(got - ref)) < tol
    lat.close()


@pytest.mark.parametrize("storage,tol", [("f32", 1e-7), ("f64", 1e-14)])
def test_fused_run_with_solids_matches_oracle(storage, tol):
    dims, walls = (37, 14, 9), (0, 1, 0)
    g, f0 = _start_walls(dims, walls, 51)
    field = workloads.gaussian_force(dims, 1e-4, 52)
    solid = workloads.random_solids(dims, 0.15, 53)
    from paper_1801_04586_amd import Lattice

    lat = Lattice(dims, walls, storage, RATES, force=(1e-5, -3e-6, 2e-6), force_field=field, solid=solid)
    lat.set_fused_steps(True)
    assert lat.uses_fused_pairs
    lat.set_populations(torch.from_numpy(f0))
    start = lat.populations().cpu().numpy()
    lat.step(4)
    got = lat.populations().cpu().numpy()
    ref = oracle.run(g, start, RATES, 4, force=(1e-5, -3e-6, 2e-6), force_field=lat.force_field.double().cpu().numpy(),
                     solid=solid)
    fl = solid == 0
    assert np.max(np.abs(got[:, fl] - ref[:, fl])) < tol
    lat.close()


@pytest.mark.parametrize("storage,tol", [("f32", 1e-7), ("f64", 1e-14)])
def test_fused_run_matches_oracle(storage, tol):
    dims = (37, 11, 6)
    g, f0 = _start(dims, 7)
    field = workloads.gaussian_force(dims, 1e-4, 8)
    from paper_1801_04586_amd import Lattice

    lat = Lattice(dims, (0, 0, 0), storage, RATES, force=(1e-5, -3e-6, 2e-6), force_field=field)
    lat.set_fused_steps(True)
    assert lat.uses_fused_pairs
    lat.set_populations(torch.from_numpy(f0))
    start = lat.populations().cpu().numpy()
    lat.step(4)
    got = lat.populations().cpu().numpy()
    ref = oracle.run(g, start, RATES, 4, force=(1e-5, -3e-6, 2e-6), force_field=lat.force_field.double().cpu().numpy())
    err = np.max(np.abs(got - ref))
    print(f"fused {storage} run against the oracle: {err:.2e}")
    assert err < tol
    lat.close()


@pytest.mark.parametrize("lattice,collision", [("d3q19", "cascaded"), ("d3q27", "mrt")])
def test_fused_fp64_d3q19_and_mrt_pairs_are_bitwise_single_steps_and_match_the_oracle(lattice, collision):
    """Periodic FP64 lattices of the D3Q19 scheme (Appendix A) and the MRT (Appendix B) in fused pairs,
    on a ragged lattice with a force field: bitwise the single steps, and within FP64 rounding of the
    oracle."""
    from paper_1801_04586_amd import Lattice

    dims = (45, 17, 9)
    q = 19 if lattice == "d3q19" else 27
    g = oracle.Geometry(dims)
    rho0, u0 = workloads.random_state_fields(dims, 111, du=0.05, drho=0.02)
    f0 = oracle.init(g, rho0, u0, lattice=lattice, model=collision) + \
        workloads.random_populations_perturbation(dims, 112, 1e-3)[:q]
    field = workloads.gaussian_force(dims, 1e-4, 113)
    out = {}
    for fused in (True, False):
        lat = Lattice(dims, (0, 0, 0), "f64", RATES, force=(1e-5, -3e-6, 2e-6), force_field=field, lattice=lattice,
                      collision=collision)
        lat.set_fused_steps(fused)
        assert lat.uses_fused_pairs == fused
        lat.set_populations(torch.from_numpy(f0))
        lat.step(5)
        out[fused] = (lat.state.clone(), lat.populations().cpu().numpy())
        lat.close()
    assert torch.equal(out[True][0], out[False][0])
    ref = oracle.run(g, f0, RATES, 5, force=(1e-5, -3e-6, 2e-6), force_field=field, lattice=lattice, model=collision)
    assert np.max(np.abs(out[True][1] - ref)) < 1e-14


@pytest.mark.parametrize("dims,walls,frac", [((67, 19, 13), (0, 0, 0), 0.0), ((45, 26, 9), (1, 1, 1), 0.2)],
                         ids=["periodic", "walls_solids"])
def test_fused_launch_writes_every_fluid_entry_and_no_padding(dims, walls, frac):
    """The output buffer of one fused launch is filled with NaN first: afterwards every fluid entry is
    finite and the plane padding is still NaN."""
    g, f0 = _start_walls(dims, walls, 101)
    solid = workloads.random_solids(dims, frac, 102) if frac else None
    from paper_1801_04586_amd import Lattice

    lat = Lattice(dims, walls, "f32", RATES, force=(1e-5, 0.0, 0.0), solid=solid)
    lat.set_fused_steps(True)
    lat.set_populations(torch.from_numpy(f0))
    lat.other.fill_(float("nan"))
    out = lat.other
    lat.step(2)
    assert lat.state.data_ptr() == out.data_ptr()
    n = int(np.prod(dims))
    body = out[:, :n].reshape((27,) + g.shape).cpu().numpy()
    fl = np.ones(g.shape, bool) if solid is None else solid == 0
    assert np.isfinite(body[:, fl]).all()
    assert torch.isnan(out[:, n:]).all()
    lat.close()


# ----------------------------------------------------------------------------- clbm_trajectory
@pytest.mark.parametrize("case", ["periodic", "walls_solids", "moving_walls", "general_rates", "fp64"])
def test_trajectory_keeps_every_state_bitwise(case):
    """clbm_trajectory stores the state after every step; where the lattice takes fused pairs, each
    launch also stores the state between its two steps.  Every kept state is bitwise the one single
    steps produce, for odd and even step counts, and the source state is left untouched."""
    from paper_1801_04586_amd import Lattice

    dims = (37, 26, 18)
    walls, solid, wv, rates, storage = (0, 0, 0), None, None, RATES_H1, "f32"
    if case == "walls_solids":
        walls, solid = (0, 1, 1), workloads.random_solids(dims, 0.15, 21)
    elif case == "moving_walls":
        walls, wv = (1, 1, 1), {(1, 1): (0.02, 0.0, -0.01), (2, 0): (0.0, 0.015, 0.0)}
    elif case == "general_rates":
        rates = RATES
    elif case == "fp64":
        storage = "f64"
    g, f0 = _start(dims, 23)
    field = workloads.gaussian_force(dims, 1e-4, 24)
    for fused in (True, False):
        lat = Lattice(dims, walls, storage, rates, force=(1e-5, 0, 0), force_field=field, solid=solid,
                      wall_velocity=wv)
        lat.set_fused_steps(fused)
        assert lat.uses_fused_pairs == fused
        lat.set_populations(torch.from_numpy(f0))
        src = lat.state.clone()
        for n in (5, 4):
            states = [lat.new_state() for _ in range(n)]
            lat.ctx.trajectory(src, states)
            a, b = src.clone(), lat.new_state()
            for k in range(n):
                lat.ctx.step(a, b)
                assert torch.equal(states[k], b), (case, fused, n, k)
                a, b = b, a
        assert torch.equal(src, lat.state)
        lat.close()


def test_trajectory_refuses_shared_buffers():
    from paper_1801_04586_amd import ClbmError, Lattice

    lat = Lattice((8, 8, 8), (0, 0, 0), "f32", RATES)
    lat.init()
    s1, s2 = lat.new_state(), lat.new_state()
    for states in ([s1, s1], [s1, lat.state], [s1, s2, s1]):
        with pytest.raises(ClbmError):
            lat.ctx.trajectory(lat.state, states)
    lat.ctx.trajectory(lat.state, [])  # nothing to do
    lat.ctx.trajectory(lat.state, [s1, s2])
    torch.cuda.synchronize()
    lat.close()


@pytest.mark.parametrize("dims,walls,frac,moving", [((67, 19, 13), (0, 0, 0), 0.0, False),
                                                    ((33, 9, 40), (1, 1, 1), 0.2, False),
                                                    ((40, 12, 3), (0, 1, 1), 0.0, False),
                                                    ((35, 13, 11), (1, 1, 1), 0.15, True),
                                                    ((38, 14, 9), (0, 1, 0), 0.0, True)])
@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_fused_mrt_pairs_are_bitwise_single_steps(dims, walls, frac, moving, storage):
    """The raw-moment MRT of Appendix B in fused pairs: periodic with a force field, walls, solids and
    moving faces, against single MRT steps."""
    g, f0 = _start_walls(dims, walls, 81)
    field = workloads.gaussian_force(dims, 1e-4, 82)
    solid = workloads.random_solids(dims, frac, 83) if frac else None
    wv = _moving_faces(walls, 84) if moving else None
    for steps in (2, 5):
        a, _ = _run_solid(dims, walls, solid, steps, True, f0, field, RATES, wv, "mrt", storage)
        b, _ = _run_solid(dims, walls, solid, steps, False, f0, field, RATES, wv, "mrt", storage)
        assert torch.equal(a, b), (dims, walls, frac, moving, steps, storage)


def _run_q19(dims, walls, solid, steps, fused, f0, field, wall_velocity=None, storage="f32"):
    from paper_1801_04586_amd import Lattice

    lat = Lattice(dims, walls, storage, RATES, force=(1e-5, -3e-6, 2e-6), force_field=field, solid=solid,
                  wall_velocity=wall_velocity, lattice="d3q19")
    lat.set_fused_steps(fused)
    assert lat.uses_fused_pairs == fused
    lat.set_populations(torch.from_numpy(f0))
    lat.step(steps)
    out = lat.state.clone()
    pops = lat.populations().cpu().numpy()
    lat.close()
    return out, pops


@pytest.mark.parametrize("dims,walls,frac,moving", [((67, 19, 13), (0, 0, 0), 0.0, False),
                                                    ((16, 8, 3), (0, 0, 0), 0.0, False),
                                                    ((33, 9, 40), (1, 1, 1), 0.2, False),
                                                    ((40, 12, 3), (0, 1, 1), 0.0, False),
                                                    ((5, 7, 2), (1, 0, 1), 0.1, False),
                                                    ((35, 13, 11), (1, 1, 1), 0.15, True),
                                                    ((38, 14, 9), (0, 1, 0), 0.0, True)])
@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_fused_d3q19_pairs_are_bitwise_single_steps(dims, walls, frac, moving, storage):
    """The D3Q19 scheme of Appendix A in fused pairs (19 planes; the corner slots hold no population),
    periodic with a force field, with walls, solids and moving faces, against single D3Q19 steps."""
    g = oracle.Geometry(dims, walls)
    rho0, u0 = workloads.random_state_fields(dims, 91, du=0.05, drho=0.02)
    f0 = oracle.init(g, rho0, u0, lattice="d3q19") + workloads.random_populations_perturbation(dims, 92, 1e-3)[:19]
    field = workloads.gaussian_force(dims, 1e-4, 93)
    solid = workloads.random_solids(dims, frac, 94) if frac else None
    wv = _moving_faces(walls, 95) if moving else None
    for steps in (2, 5):
        a, _ = _run_q19(dims, walls, solid, steps, True, f0, field, wv, storage)
        b, _ = _run_q19(dims, walls, solid, steps, False, f0, field, wv, storage)
        assert torch.equal(a, b), (dims, walls, frac, moving, steps, storage)


@pytest.mark.parametrize("storage,tol", [("f32", 5e-8), ("f64", 1e-14)])
def test_fused_d3q19_pairs_match_the_oracle(storage, tol):
    dims, walls = (37, 15, 10), (0, 1, 1)
    g = oracle.Geometry(dims, walls)
    rho0, u0 = workloads.random_state_fields(dims, 96, du=0.05, drho=0.02)
    f0 = oracle.init(g, rho0, u0, lattice="d3q19") + workloads.random_populations_perturbation(dims, 97, 1e-3)[:19]
    field = workloads.gaussian_force(dims, 1e-4, 98)
    solid = workloads.random_solids(dims, 0.1, 99)
    _, got = _run_q19(dims, walls, solid, 4, True, f0, field, storage=storage)
    ref = oracle.run(g, f0, RATES, 4, force=(1e-5, -3e-6, 2e-6), force_field=field, solid=solid, lattice="d3q19")
    fl = solid == 0
    assert np.max(np.abs(got[:, fl] - ref[:, fl])) < tol
