"""Pins of the oracle's D3Q19 cascaded LBM (Appendix A) against what the paper
and the mathematics fix: the printed transformation matrix Eq. (A4), textbook
D3Q19 weights, moments of the equilibrium summed over the velocities (not
through the oracle's matrices), conservation laws, the relaxation block of
Eq. (A3), and closed-form channel and shear-wave flows (Sec. III)."""
from __future__ import annotations

import os

import numpy as np
import pytest

import analytic
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
CS2 = 1.0 / 3.0
RATES = np.array([1.0, 1.0, 1.6, 1.2, 1.3, 0.9, 1.1, 1.25, 0.95, 1.05])


def _printed_A4():
    rows = []
    with open(os.path.join(GOLDEN, "eqA4_M_d3q19.txt")) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([int(v) for v in line.split()])
    return np.array(rows, dtype=np.int64)


def test_velocities_are_d3q19_and_the_first_19_of_d3q27(orc):
    """Eq. (A1): rest, 6 faces, 12 edges; the same vectors in the same order as Eq. (1)."""
    e = orc.q19_velocities()
    assert e.shape == (19, 3)
    assert len({tuple(v) for v in e}) == 19
    assert np.abs(e).sum(axis=1).tolist() == [0] + [1] * 6 + [2] * 12
    assert np.array_equal(e, orc.velocities()[:19])


def test_moment_set_is_closed_under_lowering_exponents(orc):
    """Eq. (A2) (slot 9 read as k_002): the 19 exponent triples with at least one zero,
    a set that contains every triple below each member, so the shift N is internal to it."""
    p = orc.q19_exponents()
    s = {tuple(v) for v in p}
    assert s == {(a, b, c) for a in range(3) for b in range(3) for c in range(3) if 0 in (a, b, c)}
    for m, n, q in s:
        for a in range(m + 1):
            for b in range(n + 1):
                for c in range(q + 1):
                    assert (a, b, c) in s


def test_M_matches_printed_eq_A4(orc):
    printed = _printed_A4()
    assert printed.shape == (19, 19)
    assert np.array_equal(orc.q19_matrix_M(), printed.astype(float))


def test_Minv_and_N(orc):
    M, Mi = orc.q19_matrix_M(), orc.q19_matrix_Minv()
    assert np.max(np.abs(M @ Mi - np.eye(19))) < 1e-14
    u = np.array([0.11, -0.07, 0.05])
    N, Nm = orc.q19_matrix_N(u), orc.q19_matrix_N(-u)
    assert np.max(np.abs(N @ Nm - np.eye(19))) < 1e-15
    p = orc.q19_exponents()
    for a in range(19):
        for b in range(19):
            if N[a, b] != 0.0:
                assert (p[b] <= p[a]).all()  # a central moment needs only raw moments below it
    # central moments by their definition equal the shift of the raw moments (Eq. (4))
    assert np.max(np.abs(orc.q19_matrix_K(u) - N @ M)) < 1e-15


def test_equilibrium_at_rest_is_textbook_d3q19(orc):
    feq = orc.q19_equilibrium(1.0, [0.0, 0.0, 0.0])
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    assert np.max(np.abs(feq - w)) < 4e-16  # one ulp of 1/3


@pytest.mark.parametrize("rho,u", [(1.0, (0.0, 0.0, 0.0)), (1.03, (0.05, -0.02, 0.08)), (0.97, (-0.1, 0.1, 0.03))])
def test_equilibrium_moments_summed_over_velocities(orc, rho, u):
    """Eq. (A5): the generalized equilibrium has density rho, momentum rho u, second moments
    rho (u u + c_s^2 I), zero central third moments in the set and central fourth moments
    rho c_s^4, all summed directly over the 19 velocities."""
    u = np.array(u)
    e = orc.q19_velocities().astype(float)
    f = orc.q19_equilibrium(rho, u)
    assert abs(f.sum() - rho) < 1e-15
    assert np.max(np.abs(f @ e - rho * u)) < 1e-15
    second = np.einsum("i,ia,ib->ab", f, e, e)
    assert np.max(np.abs(second - rho * (np.outer(u, u) + CS2 * np.eye(3)))) < 1e-15
    c = e - u
    for m, n, q in [(1, 2, 0), (1, 0, 2), (2, 1, 0), (2, 0, 1), (0, 1, 2), (0, 2, 1)]:
        assert abs(np.sum(f * c[:, 0] ** m * c[:, 1] ** n * c[:, 2] ** q)) < 1e-15
    for m, n, q in [(2, 2, 0), (2, 0, 2), (0, 2, 2)]:
        assert abs(np.sum(f * c[:, 0] ** m * c[:, 1] ** n * c[:, 2] ** q) - rho * CS2 ** 2) < 1e-15


def test_collision_conserves_mass_adds_force_and_ignores_s0_s1(orc):
    rng = np.random.default_rng(7)
    e = orc.q19_velocities().astype(float)
    for _ in range(5):
        f = orc.q19_equilibrium(1.0 + 0.02 * rng.standard_normal(), 0.05 * rng.standard_normal(3))
        f = f + 1e-3 * rng.standard_normal(19)
        F = 1e-4 * rng.standard_normal(3)
        fs = orc.q19_collide(f, F, RATES)
        assert abs(fs.sum() - f.sum()) < 1e-15
        assert np.max(np.abs(fs @ e - (f @ e + F))) < 1e-15
        other = RATES.copy()
        other[0], other[1] = 1.7, 0.4
        assert np.max(np.abs(orc.q19_collide(f, F, other) - fs)) < 1e-15
        # s3b, s4b, s5, s6 have no moment on this lattice
        other = RATES.copy()
        other[[5, 7, 8, 9]] = (1.9, 0.3, 1.4, 0.6)
        assert np.array_equal(orc.q19_collide(f, F, other), fs)


def test_relaxation_block_separates_trace_and_deviators(orc):
    """Eq. (A3): the block acts as s2b on the trace of (k200, k020, k002) and as s2 on deviators."""
    S = orc.q19_matrix_S(RATES)[7:10, 7:10]
    assert np.allclose(S @ np.ones(3), RATES[3] * np.ones(3), atol=1e-15)
    for d in (np.array([1.0, -1.0, 0.0]), np.array([1.0, 1.0, -2.0])):
        assert np.allclose(S @ d, RATES[2] * d, atol=1e-15)


def test_equilibrium_is_a_fixed_point_and_mass_is_conserved_with_walls_and_solids(orc):
    dims = (6, 5, 7)
    g = orc.Geometry(dims)
    f0 = orc.init(g, 1.01 * np.ones(g.shape), np.broadcast_to(np.array([0.03, -0.01, 0.02])[:, None, None, None],
                                                                (3,) + g.shape).copy(), lattice="d3q19")
    f1 = orc.run(g, f0, RATES, 3, lattice="d3q19")
    assert np.max(np.abs(f1 - f0)) < 1e-15
    gw = orc.Geometry(dims, (1, 0, 1))
    solid = workloads.random_solids(dims, 0.2, 3)
    rho0, u0 = workloads.random_state_fields(dims, 4)
    f = orc.init(gw, rho0, u0, lattice="d3q19")
    fl = solid == 0
    m0 = f[:, fl].sum()
    f = orc.run(gw, f, RATES, 10, force=(1e-4, 0, 0), solid=solid, lattice="d3q19")
    assert abs(f[:, fl].sum() - m0) < 1e-12 * m0


@pytest.mark.parametrize("nu", [0.1, 0.2])
def test_poiseuille_nonslip_rule_and_slip_closed_form(orc, nu):
    """Sec. III B on D3Q19: at the non-slip s3 the steady channel profile tends to the exact
    parabola as F -> 0 (residual E2 proportional to F^2, a cubic velocity term); at s3 = 1 the
    walls slip by u_s = F (16 Lambda - 3)/(24 nu) up to the same O(F^2) relative residual."""
    H = 20
    s2 = workloads.s2_from_nu(nu)
    s3n = workloads.nonslip_s3(s2)
    g = orc.Geometry((1, H, 1), (0, 1, 0))
    steps = int(20000 * 0.1 / nu)
    out = {}
    for F in (1e-5, 5e-6):
        for s3 in (s3n, 1.0):
            f = orc.run(g, orc.init(g, lattice="d3q19"), workloads.rates(nu, s3=s3), steps, force=(F, 0, 0),
                        lattice="d3q19")
            _, u = orc.macro(g, f, force=(F, 0, 0), lattice="d3q19")
            out[(F, s3)] = analytic.e2(u[0, 0, :, 0], analytic.poiseuille_steady(H, F, nu))
    assert out[(5e-6, s3n)] < 1e-8
    assert abs(out[(1e-5, s3n)] / out[(5e-6, s3n)] - 4.0) < 0.1
    lam = (1 / s2 - 0.5) * (1 / 1.0 - 0.5)
    for F in (1e-5, 5e-6):
        ua = analytic.poiseuille_steady(H, F, nu)
        pred = abs(F * (16 * lam - 3) / (24 * nu)) * np.sqrt(H / np.sum(ua ** 2))
        assert abs(out[(F, 1.0)] / pred - 1.0) < 5e-5


def test_shear_wave_viscosity(orc):
    """Sec. III A on D3Q19: decay of a shear wave at nu = 0.05 gives nu within 0.1%."""
    ny, nu, A = 101, 0.05, 1e-3
    g = orc.Geometry((1, ny, 1))
    phi = 2 * np.pi / ny
    y = np.arange(ny)
    u0 = np.zeros((3, 1, ny, 1))
    u0[0, 0, :, 0] = A * np.sin(phi * y)
    f = orc.init(g, None, u0, lattice="d3q19")
    T = int(round(2.0 / (phi * phi * nu)))
    r = workloads.rates(nu)
    f = orc.run(g, f, r, T // 10, lattice="d3q19")
    amps = []
    for _ in range(2):
        _, u = orc.macro(g, f, lattice="d3q19")
        amps.append(2 * abs(np.sum(u[0, 0, :, 0] * np.exp(-1j * phi * y))) / ny)
        f = orc.run(g, f, r, T // 2, lattice="d3q19")
    measured = np.log(amps[0] / amps[1]) / (phi * phi * (T // 2))
    assert abs(measured / nu - 1) < 1e-3
