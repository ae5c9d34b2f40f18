"""The raw-moment MRT of Appendix B and moving-wall bounce-back on the HIP path
(through the C ABI) against the oracle: initial state, steps with walls,
solids, moving faces (edges and corners included) and all storage types;
Couette flow; fused pairs; and the lid-driven cavity of Appendix B at Re = 400
(structure of the flow, and the cascaded scheme and the MRT side by side)."""
from __future__ import annotations

import itertools

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

RATES = np.array([1.0, 1.0, 1.6, 1.2, 1.3, 0.9, 1.1, 1.25, 0.95, 1.05])
TOL = {"f64": 1e-13, "f32": 5e-8, "f16": 1e-5, "bf16": 8e-5}


def _lattice(dims, walls, storage, collision="mrt", rates=RATES, force=(0.0, 0.0, 0.0), field=None, solid=None,
             wall_velocity=None):
    from paper_1801_04586_amd import Lattice

    return Lattice(dims, walls, storage, rates, force=force, force_field=field, solid=solid, collision=collision,
                   wall_velocity=wall_velocity)


def _moving(walls, seed):
    """Random velocities on the faces of the walled axes."""
    rng = np.random.default_rng(seed)
    return {(a, s): tuple(0.05 * rng.standard_normal(3)) for a in range(3) if walls[a] for s in (0, 1)}


def _compare(dims, walls, storage, steps, seed, collision="mrt", solid_frac=0.0, with_field=True, moving=False,
             force=(2e-5, -1e-5, 3e-6)):
    solid = workloads.random_solids(dims, solid_frac, seed + 5) if solid_frac else None
    g = oracle.Geometry(dims, walls)
    rho0, u0 = workloads.random_state_fields(dims, seed, du=0.05, drho=0.02)
    model = "mrt" if collision == "mrt" else "cascaded"
    f0 = oracle.init(g, rho0, u0, model=model) + workloads.random_populations_perturbation(dims, seed + 1, 1e-3)
    field = workloads.gaussian_force(dims, 1e-4, seed + 2) if with_field else None
    wv = _moving(walls, seed + 3) if moving else None
    lat = _lattice(dims, walls, storage, collision, force=force, field=field, solid=solid, wall_velocity=wv)
    lat.set_populations(torch.from_numpy(f0))
    start = lat.populations().cpu().numpy()
    fl = np.ones(g.shape, bool) if solid is None else solid == 0
    ref = oracle.run(g, start, RATES, steps, force=force, force_field=field, solid=solid, model=model,
                     wall_velocity=wv)
    lat.step(steps)
    got = lat.populations().cpu().numpy()
    lat.close()
    return np.max(np.abs(got[:, fl] - ref[:, fl]))


def test_mrt_init_is_the_discrete_equilibrium():
    dims, walls = (9, 8, 7), (0, 1, 1)
    rho0, u0 = workloads.random_state_fields(dims, 3)
    g = oracle.Geometry(dims, walls)
    ref = oracle.init(g, rho0, u0, model="mrt")
    for storage, tol in (("f64", 1e-15), ("f32", 1e-9)):
        lat = _lattice(dims, walls, storage)
        lat.init(rho0, u0)
        assert np.max(np.abs(lat.populations().cpu().numpy() - ref)) < tol, storage
        lat.close()


@pytest.mark.parametrize("walls", list(itertools.product((0, 1), repeat=3)))
def test_mrt_step_parity_f64_every_wall_combination(walls):
    assert _compare((5, 7, 3), walls, "f64", 1, 11) < TOL["f64"]
    assert _compare((5, 7, 3), walls, "f64", 8, 12, solid_frac=0.15) < TOL["f64"]


def test_mrt_step_parity_f64_several_blocks_and_ragged_tail():
    assert _compare((23, 19, 13), (0, 1, 0), "f64", 6, 31, solid_frac=0.1) < TOL["f64"]
    assert _compare((23, 19, 13), (0, 0, 0), "f64", 6, 32, with_field=False) < TOL["f64"]


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("walls,solid_frac", [((0, 0, 0), 0.0), ((1, 0, 1), 0.2)])
def test_mrt_step_parity_reduced_storage_one_step(storage, walls, solid_frac):
    assert _compare((13, 9, 7), walls, storage, 1, 41, solid_frac=solid_frac) < TOL[storage]


def test_mrt_step_parity_f32_ten_steps():
    assert _compare((13, 9, 7), (0, 1, 0), "f32", 10, 43, solid_frac=0.1) < 2e-7


@pytest.mark.parametrize("collision", ["cascaded", "mrt"])
@pytest.mark.parametrize("walls", [(0, 1, 0), (1, 1, 0), (1, 1, 1)])
def test_moving_walls_parity_f64(collision, walls):
    """Every face of every walled axis moves (random velocities), so edge and corner links cross
    two or three moving faces."""
    assert _compare((6, 5, 7), walls, "f64", 6, 51, collision=collision, moving=True) < TOL["f64"]
    assert _compare((6, 5, 7), walls, "f64", 6, 52, collision=collision, moving=True, solid_frac=0.15) < TOL["f64"]


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_moving_walls_parity_reduced_storage(storage):
    assert _compare((9, 8, 7), (1, 1, 1), storage, 1, 61, collision="cascaded", moving=True) < TOL[storage]


def test_populations_round_trip_with_moving_walls():
    dims, walls = (6, 5, 4), (1, 1, 1)
    g = oracle.Geometry(dims, walls)
    f0 = oracle.init(g) + workloads.random_populations_perturbation(dims, 71, 1e-3)
    lat = _lattice(dims, walls, "f64", "cascaded", wall_velocity=_moving(walls, 72))
    lat.set_populations(torch.from_numpy(f0))
    assert np.max(np.abs(lat.populations().cpu().numpy() - f0)) < 1e-16
    lat.close()


@pytest.mark.parametrize("collision,tol", [("cascaded", 1e-13), ("mrt", 1e-8)])
def test_couette_flow(collision, tol):
    H, U = 16, 0.01
    lat = _lattice((3, H, 2), (0, 1, 0), "f64", collision, rates=workloads.rates(0.1),
                   wall_velocity={(1, 1): (U, 0.0, 0.0)})
    lat.init()
    lat.step(8000)
    u = lat.moments()[1].cpu().numpy()
    lat.close()
    y = np.arange(H) + 0.5
    assert np.max(np.abs(u[0] - (U * y / H)[None, :, None])) < tol
    assert np.max(np.abs(u[1:])) < 1e-14


def test_mrt_fused_option_gives_the_single_step_result():
    """FP32 MRT lattices take fused step pairs when asked (and by default on lattices that fill the
    device); the result is bitwise that of single steps."""
    dims = (33, 9, 12)
    g = oracle.Geometry(dims)
    f0 = oracle.init(g, model="mrt") + workloads.random_populations_perturbation(dims, 81, 1e-3)
    field = workloads.gaussian_force(dims, 1e-4, 82)
    out = []
    for fused in (True, False):
        lat = _lattice(dims, (0, 0, 0), "f32", field=field)
        lat.set_fused_steps(fused)
        assert lat.uses_fused_pairs == fused
        lat.set_populations(torch.from_numpy(f0))
        lat.step(5)
        out.append(lat.state.clone())
        lat.close()
    assert torch.equal(out[0], out[1])


def test_mrt_adjoint_is_refused():
    from paper_1801_04586_amd.clbm import ClbmError

    lat = _lattice((5, 4, 3), (0, 0, 0), "f32")
    lat.init()
    lam = torch.zeros((27,) + lat.shape, dtype=torch.float32, device="cuda")
    with pytest.raises(ClbmError):
        lat.ctx.adjoint_step(lat.state, lam, torch.empty_like(lam))
    lat.close()


# ----------------------------------------------------------------------------- lid-driven cavity (Appendix B)
def _cavity(collision, L=64, U=0.1, Re=400.0, steps=60000):
    nu = U * L / Re
    lat = _lattice((L, L, L), (1, 1, 1), "f64", collision, rates=workloads.rates(nu),
                   wall_velocity={(1, 1): (U, 0.0, 0.0)})
    lat.init()
    lat.step(steps - 500)
    u_prev = lat.moments()[1].cpu().numpy()
    lat.step(500)
    u = lat.moments()[1].cpu().numpy()
    lat.close()
    return u, float(np.max(np.abs(u - u_prev)))


def test_lid_driven_cavity_re400():
    """Cubic cavity L = 64, lid y = L moving with U = 0.1 along x, Re = 400 (Appendix B).  Checks what
    holds without the external benchmark data (which is not available here): a steady state, mirror
    symmetry about z = L/2, one primary vortex (u_x changes sign once along the vertical centreline,
    with a return flow below -0.1 U; u_y > 0 near x = 0 and < 0 near x = L on the horizontal
    centreline), and agreement of the cascaded scheme and the MRT to 2% of U."""
    L, U = 64, 0.1
    res = {c: _cavity(c) for c in ("cascaded", "mrt")}
    for c, (u, drift) in res.items():
        ux, uy, uz = u  # [z, y, x]
        print(f"cavity {c}: drift over 500 steps {drift:.2e}, min u_x on the vertical centreline "
              f"{ux[L // 2, :, L // 2].min() / U:.4f} U")
        assert drift < 1e-5 * U
        # mirror symmetry about the mid-plane z = L/2 (node k <-> L-1-k)
        assert np.max(np.abs(ux - ux[::-1])) < 1e-9 * U
        assert np.max(np.abs(uz + uz[::-1])) < 1e-9 * U
        # primary vortex
        cl = 0.5 * (ux[L // 2 - 1, :, L // 2 - 1] + ux[L // 2, :, L // 2])
        assert cl[-1] > 0 and cl[: L // 3].min() < -0.1 * U
        assert np.sum(np.diff(np.sign(cl)) != 0) == 1
        hc = 0.5 * (uy[L // 2, L // 2, :] + uy[L // 2 - 1, L // 2, :])
        assert hc[: L // 8].max() > 0 and hc[-L // 8:].min() < 0
        # secondary flow in the plane x = L/2: where the in-plane vorticity w_x = dw/dy - dv/dz
        # peaks in the lower half of the cavity (one peak on each side of z = L/2 by symmetry)
        v = 0.5 * (uy[:, :, L // 2 - 1] + uy[:, :, L // 2])  # [z, y]
        w = 0.5 * (uz[:, :, L // 2 - 1] + uz[:, :, L // 2])
        om = np.gradient(w, axis=1) - np.gradient(v, axis=0)
        zk, yk = np.unravel_index(np.argmax(np.abs(om[: L // 2, 1: L // 2])), (L // 2, L // 2 - 1))
        print(f"cavity {c}: x = L/2 plane, strongest in-plane vorticity of the lower half at "
              f"z = {zk + 0.5:.1f}, y = {yk + 1.5:.1f} (and mirrored)")
    diff = np.max(np.abs(res["cascaded"][0] - res["mrt"][0])) / U
    print(f"cavity: max |u_cascaded - u_mrt| = {diff:.3e} U")
    assert diff < 0.02
