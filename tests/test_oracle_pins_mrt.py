"""Pins of the oracle's non-orthogonal raw-moment MRT (Appendix B) and of its
moving-wall bounce-back against what the mathematics fixes: the textbook
discrete equilibrium and Guo forcing, the BGK special case, conservation, and
closed-form channel flows (Poiseuille with the non-slip rule of Sec. III B,
Couette flow under a moving wall)."""
from __future__ import annotations

import numpy as np
import pytest

import analytic
import workloads

CS2 = 1.0 / 3.0
RATES = np.array([1.0, 1.0, 1.6, 1.2, 1.3, 0.9, 1.1, 1.25, 0.95, 1.05])


def _weights(e):
    return np.array([{0: 8 / 27, 1: 2 / 27, 2: 1 / 54, 3: 1 / 216}[int(np.abs(v).sum())] for v in e])


def test_discrete_equilibrium_moments(orc):
    """f_D^eq (Sec. II B): weights at rest; density, momentum and second moments summed over the
    velocities equal rho, rho u and rho (u u + c_s^2 I)."""
    e = orc.velocities().astype(float)
    assert np.max(np.abs(orc.mrt_feq(1.0, [0, 0, 0]) - _weights(e))) < 1e-16
    rho, u = 1.04, np.array([0.06, -0.03, 0.02])
    f = orc.mrt_feq(rho, u)
    assert abs(f.sum() - rho) < 1e-15
    assert np.max(np.abs(f @ e - rho * u)) < 1e-15
    assert np.max(np.abs(np.einsum("i,ia,ib->ab", f, e, e) - rho * (np.outer(u, u) + CS2 * np.eye(3)))) < 1e-15


def test_guo_forcing_moments(orc):
    """R_G of Appendix B carries no mass, momentum F, and second moments u F + F u."""
    e = orc.velocities().astype(float)
    u, F = np.array([0.05, 0.01, -0.04]), np.array([1e-3, -2e-3, 5e-4])
    R = orc.mrt_guo(u, F)
    assert abs(R.sum()) < 1e-18
    assert np.max(np.abs(R @ e - F)) < 1e-18
    assert np.max(np.abs(np.einsum("i,ia,ib->ab", R, e, e) - (np.outer(u, F) + np.outer(F, u)))) < 1e-18


def test_equal_rates_give_bgk_with_guo_forcing(orc):
    """With every rate equal to s, the MRT collision is the BGK collision with Guo forcing,
    f* = f - s (f - f_D^eq) + (1 - s/2) R_G, written here from the textbook formulas."""
    e = orc.velocities().astype(float)
    w = _weights(e)
    rng = np.random.default_rng(3)
    for s in (0.7, 1.0, 1.37, 1.9):
        f = orc.mrt_feq(1.02, [0.03, -0.02, 0.05]) + 1e-3 * rng.standard_normal(27)
        F = 1e-4 * rng.standard_normal(3)
        rho = f.sum()
        u = (f @ e + F / 2) / rho
        eu = e @ u
        feq = w * rho * (1 + eu / CS2 + eu ** 2 / (2 * CS2 ** 2) - u @ u / (2 * CS2))
        RG = w * (((e - u) @ F) / CS2 + eu * (e @ F) / CS2 ** 2)
        ref = f - s * (f - feq) + (1 - s / 2) * RG
        assert np.max(np.abs(orc.mrt_collide(f, F, np.full(10, s)) - ref)) < 4e-15  # dense M, M^-1 rounding (about 10 ulp of f_0)


def test_mrt_conserves_mass_adds_force_and_ignores_s0_s1(orc):
    e = orc.velocities().astype(float)
    rng = np.random.default_rng(5)
    for _ in range(4):
        f = orc.mrt_feq(1 + 0.02 * rng.standard_normal(), 0.05 * rng.standard_normal(3))
        f = f + 1e-3 * rng.standard_normal(27)
        F = 1e-4 * rng.standard_normal(3)
        fs = orc.mrt_collide(f, F, RATES)
        assert abs(fs.sum() - f.sum()) < 1e-15
        assert np.max(np.abs(fs @ e - (f @ e + F))) < 1e-15
        other = RATES.copy()
        other[:2] = (1.8, 0.3)
        assert np.max(np.abs(orc.mrt_collide(f, F, other) - fs)) < 1e-15


def test_step_ex_reproduces_step_without_moving_walls(orc):
    dims, walls = (6, 5, 4), (0, 1, 1)
    g = orc.Geometry(dims, walls)
    rho0, u0 = workloads.random_state_fields(dims, 8)
    f = orc.init(g, rho0, u0) + workloads.random_populations_perturbation(dims, 9, 1e-3)
    solid = workloads.random_solids(dims, 0.15, 10)
    a = orc.step(g, f, RATES, force=(1e-4, 0, 0), solid=solid)
    b = orc.step(g, f, RATES, force=(1e-4, 0, 0), solid=solid, wall_velocity=np.zeros((6, 3)))
    assert np.array_equal(a[:, solid == 0], b[:, solid == 0])


@pytest.mark.parametrize("nu", [0.1, 0.2])
def test_mrt_poiseuille_nonslip_and_slip(orc, nu):
    """Sec. III B with the MRT (s2b = s2): exact parabola at the non-slip s3, uniform slip
    u_s = F (16 Lambda - 3)/(24 nu) at s3 = 1."""
    H, F = 20, 1e-5
    s2 = workloads.s2_from_nu(nu)
    g = orc.Geometry((1, H, 1), (0, 1, 0))
    ua = analytic.poiseuille_steady(H, F, nu)
    steps = int(20000 * 0.1 / nu)
    for s3 in (workloads.nonslip_s3(s2), 1.0):
        f = orc.run(g, orc.init(g, model="mrt"), workloads.rates(nu, s2b=s2, s3=s3), steps, force=(F, 0, 0),
                    model="mrt")
        _, u = orc.macro(g, f, force=(F, 0, 0))
        e2 = analytic.e2(u[0, 0, :, 0], ua)
        lam = (1 / s2 - 0.5) * (1 / s3 - 0.5)
        pred = abs(F * (16 * lam - 3) / (24 * nu)) * np.sqrt(H / np.sum(ua ** 2))
        if s3 == 1.0:
            assert abs(e2 / pred - 1) < 1e-6
        else:
            assert e2 < 1e-10


def test_couette_under_a_moving_wall(orc):
    """Plane Couette flow: the wall beyond y = H - 1 moves with U along x, the one below y = 0
    rests; the steady profile is u_x = U (j + 1/2)/H.  Exact for the cascaded scheme; for the
    MRT with the quadratic equilibrium the deviation is O(U^3) (factor 8 per halving of U).
    Global mass is conserved."""
    H = 16
    g = orc.Geometry((1, H, 1), (0, 1, 0))
    y = np.arange(H) + 0.5
    errs = {}
    for model in ("cascaded", "mrt"):
        for U in (0.02, 0.01):
            f0 = orc.init(g, model=model)
            f = orc.run(g, f0, workloads.rates(0.1), 8000, model=model, wall_velocity={(1, 1): (U, 0, 0)})
            _, u = orc.macro(g, f)
            errs[(model, U)] = np.max(np.abs(u[0, 0, :, 0] - U * y / H))
            assert np.max(np.abs(u[1:])) < 1e-14
            assert abs(f.sum() - f0.sum()) < 1e-11
    assert errs[("cascaded", 0.02)] < 1e-13 and errs[("cascaded", 0.01)] < 1e-13
    assert abs(errs[("mrt", 0.02)] / errs[("mrt", 0.01)] - 8.0) < 0.2


def test_moving_wall_momentum_exchange_single_link(orc):
    """One step on a 1x1x1 lattice walled along y, top face moving with (U, 0, W): each population
    that leaves through the top face comes back reversed with -2 w_i (e_i . u_w)/c_s^2; through
    the bottom face (at rest) unchanged."""
    g = orc.Geometry((1, 1, 1), (0, 1, 0))
    f = orc.init(g)
    U, W = 0.03, -0.02
    out = orc.step(g, f, np.ones(10), wall_velocity={(1, 1): (U, 0.0, W)})
    e = orc.velocities()
    w = _weights(e.astype(float))
    fs = orc.collide(f[:, 0, 0, 0], (0, 0, 0), np.ones(10))
    for i, v in enumerate(e):
        j = int(np.where((e == -v).all(axis=1))[0][0])  # population arriving reversed
        if v[1] == 1:
            assert abs(out[j, 0, 0, 0] - (fs[i] - 2 * w[i] * (v[0] * U + v[2] * W) / CS2)) < 1e-16
        elif v[1] == -1:
            assert out[j, 0, 0, 0] == fs[i]
