"""Pins of the oracle's rate-to-moment map (Eq. (13)), its forcing slots (Eq. (16)) and its
moving-wall bounce-back rule at edges and corners.

The relaxation and forcing tests never look at the oracle's own moment order or matrices: they
build the central-moment map K(u) of Eq. (2) here in numpy, from the exponent list of Eq. (12)
(slot 9 read as k~_002) and the velocities, and probe only the oracle's single-node collision.
Each moment is identified by its exponents, and the rate it must relax with is read from the
printed Eq. (13), transcribed below.  Ten distinct rates make every slot's rate identifiable.
"""
from __future__ import annotations

import itertools

import numpy as np
import pytest

import analytic
import workloads

CS2 = 1.0 / 3.0

# Eq. (12), in printed order, with the second k~_020 read as k~_002 (slot 9)
EQ12 = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1), (2, 0, 0), (0, 2, 0),
        (0, 0, 2), (1, 2, 0), (1, 0, 2), (2, 1, 0), (2, 0, 1), (0, 1, 2), (0, 2, 1), (1, 1, 1), (2, 2, 0),
        (2, 0, 2), (0, 2, 2), (2, 1, 1), (1, 2, 1), (1, 1, 2), (1, 2, 2), (2, 1, 2), (2, 2, 1), (2, 2, 2)]
# Eq. (13), slot by slot in the same order ("block" = the 3x3 block on k~_200, k~_020, k~_002)
EQ13 = (["s0", "s1", "s1", "s1", "s2", "s2", "s2", "block", "block", "block"] + ["s3"] * 6 + ["s3b"] + ["s4"] * 3
        + ["s4b"] * 3 + ["s5"] * 3 + ["s6"])
# Eq. (16): the forcing vector C, slot by slot in the same order, as (component, power of c_s^2)
EQ16 = {1: (0, 0), 2: (1, 0), 3: (2, 0), 10: (0, 1), 11: (0, 1), 12: (1, 1), 13: (2, 1), 14: (1, 1), 15: (2, 1),
        23: (0, 2), 24: (1, 2), 25: (2, 2)}
RATE_INDEX = {name: k for k, name in enumerate(("s0", "s1", "s2", "s2b", "s3", "s3b", "s4", "s4b", "s5", "s6"))}
# ten distinct rates, none equal to 1
RATES = np.array([0.61, 0.73, 1.37, 0.83, 1.21, 0.91, 1.13, 1.46, 0.97, 1.29])


def test_transcriptions_are_consistent():
    """The transcribed lists have 27 entries, Eq. (12) is the full set {0,1,2}^3, and every moment of a
    given kind in Eq. (13) shares its order (conserved, second, third, fourth, fifth, sixth)."""
    assert len(EQ12) == 27 and len(EQ13) == 27 and len(set(EQ12)) == 27
    assert set(EQ12) == set(itertools.product(range(3), repeat=3))
    order_of = {"s0": 0, "s1": 1, "s2": 2, "block": 2, "s3": 3, "s3b": 3, "s4": 4, "s4b": 4, "s5": 5, "s6": 6}
    for p, r in zip(EQ12, EQ13):
        assert sum(p) == order_of[r], (p, r)


def _K(e, u):
    """Central-moment map of Eq. (2): K[a, i] = prod_alpha (e_i,alpha - u_alpha)^p_a,alpha, moments in
    the transcribed Eq. (12) order."""
    d = e.astype(np.float64) - np.asarray(u, dtype=np.float64)[None, :]
    P = np.array(EQ12)
    return np.prod(d[None, :, :] ** P[:, None, :], axis=2)


def _teq(rho):
    """Eq. (15) in the transcribed order: rho c_s^(m+n+p) when every exponent is even, else 0."""
    return np.array([rho * CS2 ** (sum(p) // 2) if all(v % 2 == 0 for v in p) else 0.0 for p in EQ12])


def _S(s):
    """Eq. (13) from the transcription, with s_+ = (s2b + 2 s2)/3 and s_- = (s2b - s2)/3."""
    S = np.zeros((27, 27))
    for a, name in enumerate(EQ13):
        if name != "block":
            S[a, a] = s[RATE_INDEX[name]]
    sp = (s[RATE_INDEX["s2b"]] + 2 * s[RATE_INDEX["s2"]]) / 3
    sm = (s[RATE_INDEX["s2b"]] - s[RATE_INDEX["s2"]]) / 3
    for r in range(7, 10):
        for c in range(7, 10):
            S[r, c] = sp if r == c else sm
    return S


@pytest.mark.parametrize("u", [(0.0, 0.0, 0.0), (0.05, -0.03, 0.02)])
def test_each_central_moment_relaxes_with_its_eq13_rate(orc, u):
    """Eq. (5), (13): perturb one central moment of an equilibrium by eps (f = f_eq + eps K(u)^-1 e_a,
    which leaves rho and u unchanged for a >= 4); after the oracle's collision (F = 0) the central
    moments about u deviate from T~eq by (I - S) eps e_a, with S from the printed Eq. (13).  With ten
    distinct rates this fixes the rate of every one of the 23 non-conserved moments."""
    e = orc.velocities()
    rho = 1.02
    K = _K(e, u)
    Kinv = np.linalg.inv(K)
    teq = _teq(rho)
    feq = Kinv @ teq
    S = _S(RATES)
    eps = 1e-3
    for a in range(4, 27):
        f = feq + eps * (Kinv @ np.eye(27)[a])
        fs = orc.collide(f, [0.0, 0.0, 0.0], RATES)
        got = (K @ fs - teq) / eps
        want = (np.eye(27) - S)[:, a]
        assert np.max(np.abs(got - want)) < 1e-9, (EQ12[a], EQ13[a], got[a], want[a])


def test_forcing_enters_each_eq16_slot_with_half_its_rate(orc):
    """Eq. (5), (16): from a state whose central moments about u (Eq. (9)) equal T~eq except the first
    ones, -F/2, the collision gives T~* = T~eq + (I - S/2) C, with C the printed Eq. (16); the first
    central moments become F/2 whatever s1 (Sec. II)."""
    e = orc.velocities()
    rho, u = 0.97, np.array([0.04, -0.02, 0.03])
    F = np.array([2e-3, -3e-3, 1.5e-3])
    K = _K(e, u)
    T = _teq(rho)
    T[1:4] = -F / 2
    f = np.linalg.solve(K, T)
    fs = orc.collide(f, F, RATES)
    got = K @ fs - _teq(rho)
    C = np.zeros(27)
    for a, (comp, pw) in EQ16.items():
        C[a] = F[comp] * CS2 ** pw
    want = (np.eye(27) - _S(RATES) / 2) @ C
    want[1:4] = F / 2
    assert np.max(np.abs(got - want)) < 1e-14, np.max(np.abs(got - want))


# -------------------------------------------------------------------------------------------- Sec. III B, every axis
@pytest.mark.parametrize("flow,wall", [(a, b) for a in range(3) for b in range(3) if a != b])
def test_nonslip_poiseuille_in_every_orientation(orc, flow, wall):
    """Sec. III B: the steady force-driven channel flow has no slip at s3 = (16 - 8 s2)/(8 - s2).  The
    slip depends on the rate of the third-order moment with exponent 1 along the flow and 2 across the
    channel (k~_120 for flow along x, walls across y); the six orientations cover the six moments
    Eq. (13) gives s3, while s3b, s4, s4b, s5, s6 are 1 and s2b = s2."""
    H, nu, F = 16, 0.2, 1e-6
    s2 = workloads.s2_from_nu(nu)
    s = workloads.rates(nu, s2b=s2, s3=workloads.nonslip_s3(s2))
    dims, walls, force = [1, 1, 1], [0, 0, 0], [0.0, 0.0, 0.0]
    dims[wall], walls[wall], force[flow] = H, 1, F
    g = orc.Geometry(tuple(dims), tuple(walls))
    steps = int(40 * H * H / (nu * np.pi ** 2))
    f = orc.run(g, orc.init(g), s, steps, force=tuple(force))
    _, u = orc.macro(g, f, force=tuple(force))
    prof = u[flow].reshape(H)
    err = analytic.e2(prof, analytic.poiseuille_steady(H, F, nu))
    assert err < 1e-9, err
    # the same channel at s3 = 1 slips (so the test above depends on which rate the moment takes)
    f1 = orc.run(g, orc.init(g), workloads.rates(nu, s2b=s2), steps, force=tuple(force))
    _, u1 = orc.macro(g, f1, force=tuple(force))
    assert analytic.e2(u1[flow].reshape(H), analytic.poiseuille_steady(H, F, nu)) > 1e-5


# -------------------------------------------------------------------------------------------- moving walls
def _face_velocities(rng):
    return rng.uniform(-0.05, 0.05, (6, 3))


@pytest.mark.parametrize("model,lattice", [("cascaded", "d3q27"), ("mrt", "d3q27"), ("cascaded", "d3q19")])
def test_walls_moving_with_the_fluid_keep_a_uniform_flow(orc, model, lattice):
    """Bounce-back from a wall moving at u_w returns f*_i - 2 w_i (e_i . u_w)/c_s^2.  When every face moves
    with the velocity U of a uniform equilibrium at rho = 1, the correction equals f_eq,i - f_eq,opp(i) for
    the equilibria used here (U along one axis for the cascaded generalized equilibrium; any U for the
    discrete equilibrium of the MRT), so the uniform state is stationary on a box walled on every axis --
    also for links that cross two or three faces at once (edges, corners), which therefore must take
    the velocity U, i.e. the mean of the faces they cross.  The same holds on the D3Q19 lattice of
    Appendix A, whose edge links cross two faces at the box's edges."""
    dims = (4, 5, 3)
    g = orc.Geometry(dims, (1, 1, 1))
    U = np.array([0.04, 0.0, 0.0]) if model == "cascaded" else np.array([0.03, -0.02, 0.025])
    u0 = np.zeros((3,) + g.shape)
    u0[:] = U[:, None, None, None]
    f = orc.init(g, None, u0, model=model, lattice=lattice)
    wall_u = np.tile(U, (6, 1))
    s = np.array([1.0, 1.0, 1.3, 1.1, 1.2, 0.9, 1.05, 1.15, 0.95, 1.25])
    f5 = orc.run(g, f, s, 5, model=model, wall_velocity=wall_u, lattice=lattice)
    assert np.max(np.abs(f5 - f)) < 1e-15, np.max(np.abs(f5 - f))
    # with the faces at rest the same state is not stationary
    assert np.max(np.abs(orc.run(g, f, s, 1, model=model, lattice=lattice) - f)) > 1e-3


def _permute_case(orc, perm, flip, dims, f, wall_u, Ff, solid):
    """Image of a lattice state under an axis permutation (new axis b = old axis perm[b]) followed by a
    reflection of the new axes with flip[b] = 1.  Returns (dims, f, wall_u, Ff, solid) of the image."""
    e = orc.velocities() if f.shape[0] == 27 else orc.q19_velocities()
    nd = tuple(dims[perm[b]] for b in range(3))

    def vec_img(v):  # vector components of the image
        return np.array([(-1 if flip[b] else 1) * v[perm[b]] for b in range(3)])

    def field_img(a):  # a: (..., nz, ny, nx) -> axes permuted and flipped
        ax_of = {0: -1, 1: -2, 2: -3}  # lattice axis -> array axis
        lead = a.ndim - 3
        src = [lead + 3 + ax_of[perm[b]] for b in (2, 1, 0)]  # new (z, y, x) from old array axes
        out = np.transpose(a, list(range(lead)) + src)
        for b in range(3):
            if flip[b]:
                out = np.flip(out, axis=lead + 3 + ax_of[b])
        return np.ascontiguousarray(out)

    # population i -> population j with e_j = image of e_i
    idx = {tuple(v): j for j, v in enumerate(e)}
    pmap = [idx[tuple(vec_img(e[i]))] for i in range(len(e))]
    fi = field_img(f)
    fn = np.empty_like(fi)
    for i in range(len(e)):
        fn[pmap[i]] = fi[i]
    wn = np.zeros((6, 3))
    for b in range(3):
        for side in range(2):
            old_side = 1 - side if flip[b] else side
            wn[2 * b + side] = vec_img(wall_u[2 * perm[b] + old_side])
    Fn = None
    if Ff is not None:
        Fv = field_img(Ff)
        Fn = np.stack([(-1 if flip[b] else 1) * Fv[perm[b]] for b in range(3)])
    sn = None if solid is None else field_img(solid)
    return nd, fn, wn, Fn, sn


@pytest.mark.parametrize("perm,flip", [((1, 0, 2), (0, 0, 0)), ((2, 0, 1), (0, 0, 0)), ((0, 1, 2), (1, 0, 0)),
                                       ((1, 2, 0), (0, 1, 1))])
def test_moving_wall_step_commutes_with_axis_permutations_and_reflections(orc, perm, flip):
    """The scheme is symmetric under permutations and reflections of the axes (rates of Eq. (13) depend
    only on the kind of moment, Eq. (16) is symmetric).  Stepping the image of a state equals the image
    of the stepped state, with random velocities on all six faces of a box walled on every axis, solids
    and a force field.  A bounce-back rule that favoured one of the faces an edge or corner link crosses
    breaks this; the mean of the crossed faces' velocities is the symmetric rule whose weights sum to
    one (the test above)."""
    dims = (4, 5, 6)
    g = orc.Geometry(dims, (1, 1, 1))
    rho0, u0 = workloads.random_state_fields(dims, 71, du=0.03, drho=0.01)
    f = orc.init(g, rho0, u0) + workloads.random_populations_perturbation(dims, 73, 5e-4)
    rng = np.random.default_rng(79)
    wall_u = _face_velocities(rng)
    Ff = workloads.gaussian_force(dims, 1e-4, 83)
    solid = workloads.random_solids(dims, 0.1, 89)
    s = np.array([1.0, 1.0, 1.3, 1.1, 1.2, 0.9, 1.05, 1.15, 0.95, 1.25])
    f19 = orc.init(g, rho0, u0, lattice="d3q19")
    for model, lattice, f_ in (("cascaded", "d3q27", f), ("mrt", "d3q27", f), ("cascaded", "d3q19", f19)):
        out = orc.run(g, f_, s, 2, force_field=Ff, solid=solid, model=model, wall_velocity=wall_u, lattice=lattice)
        nd, fn, wn, Fn, sn = _permute_case(orc, perm, flip, dims, f_, wall_u, Ff, solid)
        gn = orc.Geometry(nd, (1, 1, 1))
        outn = orc.run(gn, fn, s, 2, force_field=Fn, solid=sn, model=model, wall_velocity=wn, lattice=lattice)
        _, want, _, _, _ = _permute_case(orc, perm, flip, dims, out, wall_u, Ff, solid)
        assert np.max(np.abs(outn - want)) < 1e-14, (model, lattice, np.max(np.abs(outn - want)))


def _lid_duct_series(a, U, y, z, nterms=2001):
    """Steady Stokes flow u_x(y, z) in the square duct 0 < y, z < a whose face y = a slides at U along x
    (the other faces at rest): u = sum over odd n of 4U/(n pi) sinh(n pi y/a)/sinh(n pi) sin(n pi z/a)."""
    Y, Z = np.meshgrid(y, z, indexing="ij")
    u = np.zeros_like(Y)
    for n in range(1, nterms + 1, 2):
        k = n * np.pi / a
        ratio = np.exp(k * (Y - a)) * (1 - np.exp(-2 * k * Y)) / (1 - np.exp(-2 * n * np.pi))
        u += 4 * U / (n * np.pi) * ratio * np.sin(k * Z)
    return u


@pytest.mark.slow
def test_lid_driven_duct_converges_to_the_series(orc):
    """A square duct (walls in y and z, periodic along x) whose face y = a slides along x: the steady
    profile converges to the Stokes series as a grows, at first order (the velocity jumps at the two
    edges where the sliding face meets resting faces; links crossing both take half the lid velocity)."""
    U, nu = 1e-4, 1.0 / 6.0
    s = workloads.rates(nu)
    errs = []
    for a in (8, 16, 32):
        g = orc.Geometry((1, a, a), (0, 1, 1))
        wall_u = np.zeros((6, 3))
        wall_u[3] = (U, 0.0, 0.0)  # face beyond y = a - 1
        steps = int(12 * a * a / (nu * np.pi ** 2))
        f = orc.run(g, orc.init(g), s, steps, wall_velocity=wall_u)
        _, u = orc.macro(g, f)
        c = np.arange(a) + 0.5
        ua = _lid_duct_series(a, U, c, c)  # indexed [y, z]
        errs.append(analytic.e2(u[0, :, :, 0].T, ua))
    # first order (the corner discontinuity): 9.5e-3, 4.6e-3, 2.3e-3
    assert errs[1] < 0.6 * errs[0] and errs[2] < 0.6 * errs[1], errs
    assert errs[2] < 3e-3, errs
