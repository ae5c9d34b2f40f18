"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of these re-types the oracle's
own formula: they compare against the printed matrix (Eq. 14), the printed
example row of N (Sec. II B), textbook D3Q27 weights and Maxwellian moments,
closed-form product forms of the equilibrium and forcing, exact rational
arithmetic, conservation laws, special cases that collapse to BGK/MRT
(Sec. II A) and closed-form flows (Sec. III).
"""
from __future__ import annotations

import os
from fractions import Fraction

import numpy as np
import pytest

import analytic
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
CS2 = 1.0 / 3.0


def _load_int_matrix(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([int(v) for v in line.split()])
    return np.array(rows, dtype=np.int64)


# -------------------------------------------------------------------------------------------- P1: M, M^-1
def test_velocity_set_is_d3q27(orc):
    """Eq. (1): 27 distinct velocities in {-1,0,1}^3, rest first, opposite pairs present."""
    e = orc.velocities()
    assert e.shape == (27, 3)
    assert len({tuple(v) for v in e}) == 27
    assert tuple(e[0]) == (0, 0, 0)
    assert np.abs(e).sum(axis=1).tolist() == [0] + [1] * 6 + [2] * 12 + [3] * 8
    for v in e:
        assert any((w == -v).all() for w in e)


def test_moment_set_is_full_tensor_set_in_ascending_order(orc):
    """Eq. (12) with slot 9 read as k_002: exactly {0,1,2}^3, ordered by ascending m+n+p."""
    p = orc.exponents()
    assert len({tuple(v) for v in p}) == 27
    assert set(map(tuple, p)) == {(a, b, c) for a in range(3) for b in range(3) for c in range(3)}
    orders = p.sum(axis=1)
    assert (np.diff(orders) >= 0).all()


def test_M_matches_printed_eq14(orc):
    """Eq. (14): M built from the definition Eq. (2)/(4) equals the printed matrix entrywise."""
    printed = _load_int_matrix("eq14_M_d3q27.txt")
    assert printed.shape == (27, 27)
    M = orc.matrix_M()
    assert np.array_equal(M, printed.astype(np.float64))


def test_nonzero_counts_of_M_and_Minv(orc):
    """Sec. II B: M and M^-1 have 343 and 216 non-zero entries."""
    M = orc.matrix_M()
    Minv = orc.matrix_Minv()
    assert np.count_nonzero(M) == 343
    assert np.count_nonzero(np.abs(Minv) > 1e-12) == 216


def test_Minv_is_exact_rational_inverse(orc):
    """M^-1 against an exact Gauss-Jordan inverse of the printed Eq. (14) in rational arithmetic."""
    printed = _load_int_matrix("eq14_M_d3q27.txt")
    n = 27
    W = [[Fraction(int(printed[r, c])) for c in range(n)] + [Fraction(int(r == c)) for c in range(n)]
         for r in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if W[r][col] != 0)
        W[col], W[piv] = W[piv], W[col]
        d = W[col][col]
        W[col] = [v / d for v in W[col]]
        for r in range(n):
            if r != col and W[r][col] != 0:
                m = W[r][col]
                W[r] = [a - m * b for a, b in zip(W[r], W[col])]
    exact = np.array([[float(W[r][n + c]) for c in range(n)] for r in range(n)])
    Minv = orc.matrix_Minv()
    assert np.max(np.abs(Minv - exact)) < 1e-14
    assert np.max(np.abs(orc.matrix_M() @ Minv - np.eye(27))) < 1e-14


# -------------------------------------------------------------------------------------------- P2: N, N^-1
def test_N_row4_matches_printed_example(orc):
    """Sec. II B: N_4 = [u_x u_y, -u_y, -u_x, 0, 1, 0, ..., 0]."""
    u = np.array([0.031, -0.047, 0.013])
    N = orc.matrix_N(u)
    expect = np.zeros(27)
    expect[0] = u[0] * u[1]
    expect[1] = -u[1]
    expect[2] = -u[0]
    expect[4] = 1.0
    assert np.max(np.abs(N[4] - expect)) < 1e-16


def test_N_is_lower_triangular_and_inverse_is_N_of_minus_u(orc):
    """Sec. II B: N is lower triangular (binomial theorem); N(u) N(-u) = I and equals a numerical inverse."""
    rng = np.random.default_rng(3)
    for _ in range(5):
        u = rng.uniform(-0.3, 0.3, 3)
        N = orc.matrix_N(u)
        assert np.max(np.abs(np.triu(N, 1))) == 0.0
        assert np.allclose(np.diag(N), 1.0)
        Ninv = orc.matrix_Ninv(u)
        assert np.max(np.abs(N @ Ninv - np.eye(27))) < 1e-14
        assert np.max(np.abs(np.linalg.inv(N) - Ninv)) < 1e-12
        assert np.count_nonzero(np.abs(N) > 0) == 216


def test_central_moment_matrix_equals_shift_times_M(orc):
    """Eq. (4): the central moments by the definition Eq. (2) equal N(u) M (two independent routes)."""
    rng = np.random.default_rng(5)
    u = rng.uniform(-0.2, 0.2, 3)
    assert np.max(np.abs(orc.matrix_K(u) - orc.matrix_N(u) @ orc.matrix_M())) < 1e-14


# -------------------------------------------------------------------------------------------- P3, P4
def _g(e, u):
    return np.where(e == 0, 2.0 / 3.0 - u * u, 0.5 * (u * u + 1.0 / 3.0 + e * u))


def _h(e, u):
    return np.where(e == 0, -2.0 * u, u + 0.5 * e)


def test_equilibrium_product_form_and_textbook_weights(orc):
    """Sec. II B: the generalized equilibrium (NM)^-1 T_eq is the product rho prod_a g(e_a, u_a);
    at u = 0 it reduces to the textbook D3Q27 weights 8/27, 2/27, 1/54, 1/216."""
    e = orc.velocities()
    w = orc.equilibrium(1.0, [0, 0, 0])
    ref = {0: 8 / 27, 1: 2 / 27, 2: 1 / 54, 3: 1 / 216}
    for i in range(27):
        assert abs(w[i] - ref[int(np.abs(e[i]).sum())]) < 4e-16
    rng = np.random.default_rng(11)
    for _ in range(5):
        rho = rng.uniform(0.9, 1.1)
        u = rng.uniform(-0.2, 0.2, 3)
        feq = orc.equilibrium(rho, u)
        prod = rho * _g(e[:, 0], u[0]) * _g(e[:, 1], u[1]) * _g(e[:, 2], u[2])
        assert np.max(np.abs(feq - prod)) < 1e-15


def test_equilibrium_has_maxwellian_moments(orc):
    """Eq. (15): mass rho, momentum rho u, momentum flux rho (c_s^2 delta + u u) of the equilibrium."""
    e = orc.velocities().astype(float)
    rho, u = 1.07, np.array([0.05, -0.02, 0.11])
    feq = orc.equilibrium(rho, u)
    assert abs(feq.sum() - rho) < 1e-15
    assert np.max(np.abs(feq @ e - rho * u)) < 1e-15
    Pi = np.einsum("i,ia,ib->ab", feq, e, e)
    assert np.max(np.abs(Pi - rho * (CS2 * np.eye(3) + np.outer(u, u)))) < 1e-15


def test_forcing_vector_product_form(orc):
    """Eq. (16): (NM)^-1 C = sum_a F_a h(e_a, u_a) prod_{b != a} g(e_b, u_b) with h(0,u) = -2u, h(+-1,u) = u +- 1/2."""
    e = orc.velocities()
    rng = np.random.default_rng(13)
    for _ in range(5):
        u = rng.uniform(-0.2, 0.2, 3)
        F = rng.normal(0, 1e-3, 3)
        L = orc.matrix_Minv() @ orc.matrix_Ninv(u)
        r = L @ orc.cvec(F)
        g = [_g(e[:, a], u[a]) for a in range(3)]
        h = [_h(e[:, a], u[a]) for a in range(3)]
        ref = F[0] * h[0] * g[1] * g[2] + F[1] * g[0] * h[1] * g[2] + F[2] * g[0] * g[1] * h[2]
        assert np.max(np.abs(r - ref)) < 1e-17


def test_printed_C_versus_exact_NMR(orc):
    """Eq. (16) reading: N M R with R of Eq. (6) on the generalized equilibrium differs from the printed C
    only by O(F u^3) terms in the second-, fourth- and sixth-order even slots."""
    rng = np.random.default_rng(17)
    e = orc.velocities().astype(float)
    for _ in range(3):
        rho = rng.uniform(0.95, 1.05)
        u = rng.uniform(-0.1, 0.1, 3)
        F = rng.normal(0, 1e-3, 3)
        feq = orc.equilibrium(rho, u)
        R = ((e - u) @ F) / (rho * CS2) * feq
        NMR = orc.matrix_N(u) @ orc.matrix_M() @ R
        d = NMR - orc.cvec(F)
        Fu3 = F * u ** 3
        expect = np.zeros(27)
        expect[7:10] = -3.0 * Fu3
        expect[17] = -(Fu3[0] + Fu3[1])
        expect[18] = -(Fu3[0] + Fu3[2])
        expect[19] = -(Fu3[1] + Fu3[2])
        expect[26] = -Fu3.sum() / 3.0
        assert np.max(np.abs(d - expect)) < 1e-17


# -------------------------------------------------------------------------------------------- P5-P9: one node
def _random_state(orc, rng, amp=2e-3):
    rho = rng.uniform(0.95, 1.05)
    u = rng.uniform(-0.1, 0.1, 3)
    return orc.equilibrium(rho, u) + rng.uniform(-amp, amp, 27)


def test_collision_conserves_mass_and_adds_force(orc):
    """Eq. (5) + Eq. (16): sum f* = sum f and sum f* e = sum f e + F at every node."""
    e = orc.velocities().astype(float)
    rng = np.random.default_rng(19)
    s = np.array([1.3, 0.7, 1.6, 1.1, 1.2, 0.9, 1.4, 1.05, 1.15, 0.85])
    for _ in range(10):
        f = _random_state(orc, rng)
        F = rng.normal(0, 1e-3, 3)
        fs = orc.collide(f, F, s)
        assert abs(fs.sum() - f.sum()) < 1e-15
        assert np.max(np.abs(fs @ e - (f @ e + F))) < 1e-15


def test_conserved_rates_have_no_effect(orc):
    """Sec. III: s0 and s1 act on conserved moments; the result does not depend on them."""
    rng = np.random.default_rng(23)
    f = _random_state(orc, rng)
    F = rng.normal(0, 1e-3, 3)
    base = np.array([1.0, 1.0, 1.6, 1.1, 1.2, 0.9, 1.4, 1.05, 1.15, 0.85])
    ref = orc.collide(f, F, base)
    for s0, s1 in [(0.3, 1.7), (1.9, 0.2), (1.5, 1.5)]:
        s = base.copy()
        s[0], s[1] = s0, s1
        assert np.max(np.abs(orc.collide(f, F, s) - ref)) < 1e-15


def test_equilibrium_is_fixed_point_without_force(orc):
    """With F = 0, f = f_eq is unchanged by the collision for any rates."""
    rng = np.random.default_rng(29)
    s = rng.uniform(0.5, 1.9, 10)
    for _ in range(5):
        feq = orc.equilibrium(rng.uniform(0.9, 1.1), rng.uniform(-0.15, 0.15, 3))
        assert np.max(np.abs(orc.collide(feq, [0, 0, 0], s) - feq)) < 1e-15


def test_equal_rates_collapse_to_bgk(orc):
    """Sec. II A: with all rates equal the scheme is SRT: f* = (1-s) f + s f_eq + (1 - s/2) R',
    with f_eq and R' = (NM)^-1 C given by their product forms (independent of M and N)."""
    e = orc.velocities()
    rng = np.random.default_rng(31)
    for s_ in (0.6, 1.0, 1.7):
        f = _random_state(orc, rng)
        F = rng.normal(0, 1e-3, 3)
        rho = f.sum()
        u = (f @ e + 0.5 * F) / rho
        g = [_g(e[:, a], u[a]) for a in range(3)]
        h = [_h(e[:, a], u[a]) for a in range(3)]
        feq = rho * g[0] * g[1] * g[2]
        Rp = F[0] * h[0] * g[1] * g[2] + F[1] * g[0] * h[1] * g[2] + F[2] * g[0] * g[1] * h[2]
        ref = (1 - s_) * f + s_ * feq + (1 - s_ / 2) * Rp
        assert np.max(np.abs(orc.collide(f, F, np.full(10, s_)) - ref)) < 1e-15


def test_zero_velocity_collapses_to_raw_moment_mrt(orc):
    """Sec. II A: with N = I (u = 0) the scheme is an MRT on the raw moments of Eq. (12)."""
    rng = np.random.default_rng(37)
    M = orc.matrix_M()
    Minv = np.linalg.inv(M)
    s = rng.uniform(0.5, 1.9, 10)
    f = orc.equilibrium(1.02, [0, 0, 0]) + rng.uniform(-1e-3, 1e-3, 27)
    # remove momentum so that u = 0 exactly (F = 0): symmetrise f_i and f_opp(i)
    e = orc.velocities()
    opp = [int(np.where((e == -e[i]).all(axis=1))[0][0]) for i in range(27)]
    f = 0.5 * (f + f[opp])
    S = orc.matrix_S(s)
    teq = np.zeros(27)
    teq[0] = f.sum()
    teq[7:10] = f.sum() / 3.0
    teq[17:20] = f.sum() / 9.0
    teq[26] = f.sum() / 27.0
    ref = Minv @ ((np.eye(27) - S) @ (M @ f) + S @ teq)
    assert np.max(np.abs(orc.collide(f, [0, 0, 0], s) - ref)) < 1e-15


def test_relaxation_block_separates_trace_and_deviator(orc):
    """Eq. (13): the 3x3 block relaxes the trace at s2b and traceless parts at s2."""
    s = np.array([1, 1, 1.6, 0.7, 1, 1, 1, 1, 1, 1.0])
    B = orc.matrix_S(s)[7:10, 7:10]
    assert np.allclose(B @ np.ones(3), 0.7 * np.ones(3), atol=1e-15)
    for v in (np.array([1.0, -1.0, 0.0]), np.array([1.0, 1.0, -2.0])):
        assert np.allclose(B @ v, 1.6 * v, atol=1e-15)


# -------------------------------------------------------------------------------------------- lattice invariants
def test_streaming_conserves_mass_and_periodic_momentum_grows_by_force(orc):
    """Eq. (8)-(9): half-way bounce-back and periodic streaming conserve mass; on an all-periodic
    lattice total momentum grows by sum_x F per step."""
    dims = (5, 4, 3)
    g = orc.Geometry(dims, (0, 0, 0))
    rho0, u0 = workloads.random_state_fields(dims, 41)
    f = orc.init(g, rho0, u0) + workloads.random_populations_perturbation(dims, 43, 1e-3)
    Ff = workloads.gaussian_force(dims, 1e-4, 47)
    e = orc.velocities().astype(float)
    s = workloads.rates(0.07)
    m0 = f.sum()
    p0 = np.einsum("iz...,ia->a", f.reshape(27, -1), e)
    f1 = orc.step(g, f, s, force_field=Ff)
    assert abs(f1.sum() - m0) < 1e-12 * m0
    p1 = np.einsum("iz...,ia->a", f1.reshape(27, -1), e)
    assert np.max(np.abs(p1 - p0 - Ff.reshape(3, -1).sum(axis=1))) < 1e-14

    gw = orc.Geometry(dims, (1, 1, 1))
    solid = workloads.random_solids(dims, 0.2, 53)
    f2 = orc.step(gw, f, s, force_field=Ff, solid=solid)
    assert abs(f2.sum() - m0) < 1e-12 * m0


def test_uniform_equilibrium_is_fixed_point_of_step(orc):
    """Without force, a uniform equilibrium on a periodic lattice is stationary."""
    dims = (3, 4, 2)
    g = orc.Geometry(dims)
    rho0 = np.full((2, 4, 3), 1.03)
    u0 = np.zeros((3, 2, 4, 3))
    u0[0], u0[1], u0[2] = 0.04, -0.02, 0.01
    f = orc.init(g, rho0, u0)
    f5 = orc.run(g, f, workloads.rates(0.02), 5)
    assert np.max(np.abs(f5 - f)) < 1e-15


def test_window_matches_full_lattice_inside_the_cone(orc):
    """A window of half-width k around a node reproduces the full-lattice result at its centre after k steps."""
    dims = (9, 10, 11)
    walls = (0, 1, 0)
    full = orc.Geometry(dims, walls)
    rho0, u0 = workloads.random_state_fields(dims, 59)
    f = orc.init(full, rho0, u0) + workloads.random_populations_perturbation(dims, 61, 1e-3)
    Ff = workloads.gaussian_force(dims, 1e-4, 67)
    solid = workloads.random_solids(dims, 0.15, 71)
    s = workloads.rates(0.05)
    k = 2
    ref = orc.run(full, f, s, k, force_field=Ff, solid=solid)
    for cx, cy, cz in [(4, 5, 5), (0, 2, 10), (8, 7, 0)]:
        o = (cx - k, cy - k, cz - k)
        w = (2 * k + 1,) * 3
        g = orc.Geometry(dims, walls, o, w)
        zi = np.arange(o[2], o[2] + w[2]) % dims[2]
        yi = np.arange(o[1], o[1] + w[1]) % dims[1]
        xi = np.arange(o[0], o[0] + w[0]) % dims[0]
        sub = lambda a: np.ascontiguousarray(a[..., zi[:, None, None], yi[None, :, None], xi[None, None, :]])
        if walls[1] and (o[1] < 0 or o[1] + w[1] > dims[1]):
            continue
        fw = orc.run(g, sub(f), s, k, force_field=sub(Ff), solid=sub(solid))
        assert np.max(np.abs(fw[:, k, k, k] - ref[:, cz, cy, cx])) == 0.0


# -------------------------------------------------------------------------------------------- P10, P11: Poiseuille
@pytest.mark.parametrize("H,nu", [(20, 0.1), (16, 0.2)])
def test_poiseuille_nonslip_rule_gives_exact_parabola(orc, H, nu):
    """Sec. III B: with s3 = (16 - 8 s2)/(8 - s2) the steady Poiseuille profile has no slip:
    E2 against the parabola is at round-off level (run to steady state)."""
    F = 1e-6
    s2 = workloads.s2_from_nu(nu)
    s = workloads.rates(nu, s3=workloads.nonslip_s3(s2))
    g = orc.Geometry((1, H, 1), (0, 1, 0))
    f = orc.init(g)
    steps = int(40 * H * H / (nu * np.pi ** 2))
    f = orc.run(g, f, s, steps, force=(F, 0, 0))
    _, u = orc.macro(g, f, force=(F, 0, 0))
    err = analytic.e2(u[0, 0, :, 0], analytic.poiseuille_steady(H, F, nu))
    assert err < 1e-9, err


def test_poiseuille_other_s3_slips_by_the_closed_form_amount(orc):
    """Sec. III B (Fig. 2b): away from the non-slip rule the steady profile slips.  The slip is uniform,
    u_s = F (16 Lambda - 3) / (24 nu) with Lambda = (1/s2 - 1/2)(1/s3 - 1/2), which vanishes exactly
    on the rule (Lambda = 3/16); the profile equals parabola + u_s to round-off."""
    H, nu, F = 20, 0.1, 1e-6
    s2, s3 = workloads.s2_from_nu(nu), 1.0
    s = workloads.rates(nu, s3=s3)
    g = orc.Geometry((1, H, 1), (0, 1, 0))
    f = orc.run(g, orc.init(g), s, int(40 * H * H / (nu * np.pi ** 2)), force=(F, 0, 0))
    _, u = orc.macro(g, f, force=(F, 0, 0))
    ua = analytic.poiseuille_steady(H, F, nu)
    err = analytic.e2(u[0, 0, :, 0], ua)
    assert 1e-5 < err < 1e-2, err
    lam = (1.0 / s2 - 0.5) * (1.0 / s3 - 0.5)
    us = F * (16.0 * lam - 3.0) / (24.0 * nu)
    assert analytic.e2(u[0, 0, :, 0], ua + us) < 1e-9


def test_poiseuille_startup_3000_steps(orc):
    """Channel of 32 nodes, nu = 0.1, F = 1e-6, 3000 steps from rest against the start-up series."""
    H, nu, F, T = 32, 0.1, 1e-6, 3000
    g = orc.Geometry((1, H, 1), (0, 1, 0))
    s_ns = workloads.rates(nu, s3=workloads.nonslip_s3(workloads.s2_from_nu(nu)))
    f = orc.run(g, orc.init(g), s_ns, T, force=(F, 0, 0))
    _, u = orc.macro(g, f, force=(F, 0, 0))
    err = analytic.e2(u[0, 0, :, 0], analytic.poiseuille_startup(H, F, nu, T))
    assert err < 5e-5, err
    f1 = orc.run(g, orc.init(g), workloads.rates(nu), T, force=(F, 0, 0))
    _, u1 = orc.macro(g, f1, force=(F, 0, 0))
    err1 = analytic.e2(u1[0, 0, :, 0], analytic.poiseuille_startup(H, F, nu, T))
    assert err1 < 2e-3, err1


# -------------------------------------------------------------------------------------------- adjoint (P17)
def _adj_case(orc, dims=(4, 5, 3), walls=(0, 1, 0), solid_frac=0.0, seed=101):
    g = orc.Geometry(dims, walls)
    rho0, u0 = workloads.random_state_fields(dims, seed, du=0.03, drho=0.01)
    f0 = orc.init(g, rho0, u0) + workloads.random_populations_perturbation(dims, seed + 1, 5e-4)
    Ff = workloads.gaussian_force(dims, 1e-4, seed + 2)
    solid = workloads.random_solids(dims, solid_frac, seed + 3) if solid_frac else None
    ut = workloads.uniform_random_velocity(dims, 0.02, seed + 4)
    s = np.array([1.0, 1.0, 1.55, 1.2, 1.3, 0.9, 1.1, 1.25, 0.95, 1.05])
    return g, f0, Ff, solid, ut, s


def _J(orc, g, f0, s, T, ut, Ff, solid):
    f = orc.run(g, f0, s, T, force_field=Ff, solid=solid)
    J, _, _ = orc.loss_seed(g, f, ut, force_field=Ff, solid=solid)
    return J


@pytest.mark.parametrize("solid_frac", [0.0, 0.2])
def test_adjoint_matches_central_differences(orc, solid_frac):
    """Exact discrete adjoint against central finite differences of the forward oracle (FP64)."""
    g, f0, Ff, solid, ut, s = _adj_case(orc, solid_frac=solid_frac)
    T = 3
    J, gF, gs, gf0 = orc.loss_and_grads(g, f0, s, T, ut, force_field=Ff, solid=solid)
    rng = np.random.default_rng(7)
    fluid = 1.0 if solid is None else (1 - solid)[None].astype(float)
    # force-field direction
    v = rng.normal(0, 1, Ff.shape) * fluid
    eps = 1e-6
    fd = (_J(orc, g, f0, s, T, ut, Ff + eps * v, solid) - _J(orc, g, f0, s, T, ut, Ff - eps * v, solid)) / (2 * eps)
    assert abs(fd - np.sum(gF * v)) <= 1e-6 * abs(fd) + 1e-14
    # initial-population direction
    w = rng.normal(0, 1, f0.shape) * fluid
    eps = 1e-7
    fd = (_J(orc, g, f0 + eps * w, s, T, ut, Ff, solid) - _J(orc, g, f0 - eps * w, s, T, ut, Ff, solid)) / (2 * eps)
    assert abs(fd - np.sum(gf0 * w)) <= 1e-6 * abs(fd) + 1e-14
    # each non-conserved rate
    for k in range(2, 10):
        sp, sm = s.copy(), s.copy()
        sp[k] += 1e-4
        sm[k] -= 1e-4
        fd = (_J(orc, g, f0, sp, T, ut, Ff, solid) - _J(orc, g, f0, sm, T, ut, Ff, solid)) / 2e-4
        assert abs(fd - gs[k]) <= 1e-6 * abs(fd) + 1e-9 * np.max(np.abs(gs)), (k, fd, gs[k])
    # conserved rates have no influence
    assert abs(gs[0]) < 1e-14 and abs(gs[1]) < 1e-11 * np.max(np.abs(gs[2:]))


def test_adjoint_step_dot_product(orc):
    """<w, (dStep/df) v> = <(dStep/df)^T w, v> for one step, with the linearisation from central differences."""
    g, f0, Ff, solid, ut, s = _adj_case(orc, dims=(3, 4, 5), walls=(1, 0, 1), solid_frac=0.15, seed=202)
    rng = np.random.default_rng(9)
    fluid = (1 - solid)[None].astype(float)
    v = rng.normal(0, 1, f0.shape) * fluid
    w = rng.normal(0, 1, f0.shape) * fluid
    eps = 1e-7
    Jv = (orc.step(g, f0 + eps * v, s, force_field=Ff, solid=solid)
          - orc.step(g, f0 - eps * v, s, force_field=Ff, solid=solid)) / (2 * eps)
    lam, _, _ = orc.adjoint_step(g, f0, w, s, force_field=Ff, solid=solid)
    lhs = np.sum(w * Jv)
    rhs = np.sum(lam * v)
    assert abs(lhs - rhs) <= 1e-7 * abs(lhs)
