"""The paper's verification studies (Sec. III) run on the HIP path (FP64 unless
stated), against the closed-form flows of tests/analytic.py.

  * shear-wave decay on a moving frame, 5 x 101 x 5 (Sec. III A): the measured
    viscosity is within 0.08% of the imposed nu = 0.05 at Ma = 0.3 in the paper;
    here it is also independent of Ma (Galilean invariance of the central-moment
    equilibrium);
  * steady Poiseuille flow, 2L = 20 (Sec. III B): E2 against s3 at nu = 0.1 and
    0.2, negligible at the non-slip rule; E2 against the bulk viscosity xi,
    smallest at xi = 2 nu / 3 and linear in |xi - 2 nu / 3|;
  * square duct, a = 16 (Sec. III C): the local error E(z) against s3 at
    z = 0.5, 7.5, 12.5;
  * forced Taylor-Green vortex (Sec. III D): second-order convergence of E2 at
    T* = 4 over L = 16 ... 128 (fitted slope 2.0345 in the paper).

Each test prints what it measured (run pytest with -s to see the table).
"""
from __future__ import annotations

import numpy as np
import pytest

import analytic
import workloads

pytestmark = pytest.mark.gpu


def _lattice(dims, walls, storage, rates, **kw):
    from paper_1801_04586_amd import Lattice

    return Lattice(dims, walls, storage, rates, **kw)


def _velocity(lat):
    _, u, _, nbad = lat.moments()
    assert nbad == 0
    return u.cpu().numpy()


# ----------------------------------------------------------------------------- Sec. III A: shear wave
def _shear_wave_viscosity(Ma: float, storage: str = "f64", nu: float = 0.05, A: float = 1e-3):
    """Viscosity from the decay of the first Fourier mode of u_x(y) between t* = 0.2 and t* = 2
    (phi^2 nu t), on 5 x 101 x 5 with u = (A sin(phi y), B, 0), B = Ma c_s."""
    ny = 101
    dims = (5, ny, 5)
    phi = 2.0 * np.pi / ny
    B = Ma / np.sqrt(3.0)
    y = np.arange(ny)
    u0 = np.zeros((3, 5, ny, 5))
    u0[0] = (A * np.sin(phi * y))[None, :, None]
    u0[1] = B
    lat = _lattice(dims, (0, 0, 0), storage, workloads.rates(nu))
    lat.init(np.ones((5, ny, 5)), u0)
    T = int(round(2.0 / (phi * phi * nu)))
    marks = np.linspace(0.1 * T, T, 10).round().astype(int)
    amps, ts = [], []
    for t in marks:
        lat.step(int(t) - lat.t)
        ux = _velocity(lat)[0].mean(axis=(0, 2))
        amps.append(2.0 * abs(np.sum(ux * np.exp(-1j * phi * y))) / ny)
        ts.append(lat.t)
    lat.close()
    slope = np.polyfit(np.array(ts, float), np.log(amps), 1)[0]
    return -slope / (phi * phi)


def test_shear_wave_viscosity_is_galilean_invariant():
    nu = 0.05
    got = {Ma: _shear_wave_viscosity(Ma) for Ma in (0.0, 0.1, 0.2, 0.3)}
    for Ma, v in got.items():
        print(f"shear wave FP64 Ma={Ma:.1f}: nu = {v:.7f}, relative error {v / nu - 1:+.3e}")
    for Ma, v in got.items():
        assert abs(v / nu - 1.0) < 8e-4, (Ma, v)  # the paper's 0.08% at Ma = 0.3
        assert abs(v - got[0.0]) / nu < 1e-4, (Ma, v)  # independent of the frame velocity


def test_shear_wave_viscosity_fp32_storage():
    v = _shear_wave_viscosity(0.3, "f32")
    print(f"shear wave FP32 Ma=0.3: nu = {v:.7f}, relative error {v / 0.05 - 1:+.3e}")
    assert abs(v / 0.05 - 1.0) < 8e-4


# ----------------------------------------------------------------------------- Sec. III B: Poiseuille
H = 20


def _poiseuille_e2(nu: float, s3: float, s2b=None, steps: int = 12000):
    """Steady channel (walls in y, 2L = 20 nodes, 5 nodes along x and z), u0 = 0.05 (Re = 10 at nu = 0.1)."""
    u0 = 0.05
    F = 2.0 * nu * u0 / (H / 2) ** 2
    rates = workloads.rates(nu, s2b=s2b, s3=s3)
    lat = _lattice((5, H, 5), (0, 1, 0), "f64", rates, force=(F, 0.0, 0.0))
    lat.init()
    lat.step(steps)
    u = _velocity(lat)
    lat.step(200)
    drift = np.max(np.abs(_velocity(lat) - u))
    lat.close()
    assert drift < 1e-13 * u0  # steady
    ua = analytic.poiseuille_steady(H, F, nu)
    full = np.zeros_like(u)
    full[0] = ua[None, :, None]
    return analytic.e2(u, full), F, ua


@pytest.mark.parametrize("nu", [0.1, 0.2])
def test_poiseuille_error_against_s3_vanishes_at_the_nonslip_rule(nu):
    """With s2b = s2 (xi = 2 nu / 3, so that the bulk-viscosity error of the next test is absent)
    E2 is the uniform wall slip of the closed form, and vanishes at the non-slip s3."""
    s2 = workloads.s2_from_nu(nu)
    s3n = workloads.nonslip_s3(s2)
    steps = int(12000 * 0.1 / nu) + 4000
    rows = []
    for s3 in (0.6, 0.8, 1.0, s3n, 1.2, 1.4):
        e, F, ua = _poiseuille_e2(nu, s3, s2b=s2, steps=steps)
        lam = (1.0 / s2 - 0.5) * (1.0 / s3 - 0.5)
        slip = F * (16.0 * lam - 3.0) / (24.0 * nu)  # uniform slip of the bounce-back walls
        predicted = abs(slip) * np.sqrt(H / np.sum(ua ** 2))
        rows.append((s3, e, predicted))
        print(f"Poiseuille nu={nu}: s3={s3:.5f} E2={e:.3e} (uniform-slip prediction {predicted:.3e})")
    for s3, e, predicted in rows:
        if s3 == s3n:
            assert e < 1e-10
        else:
            assert abs(e - predicted) <= 1e-4 * predicted
    assert min(rows, key=lambda r: r[1])[0] == s3n


def test_poiseuille_error_against_bulk_viscosity():
    nu = 0.1
    s2 = workloads.s2_from_nu(nu)
    s3n = workloads.nonslip_s3(s2)
    rows = []
    # s2b above about 1.75 is linearly unstable with s2 = 1.25 and the other rates 1 (the growth
    # rate of a small perturbation at rest exceeds one), so the sweep stays below it
    for s2b in (0.6, 0.8, 1.0, s2, 1.4, 1.6):
        e, _, _ = _poiseuille_e2(nu, s3n, s2b=s2b, steps=16000)
        xi = (2.0 / 3.0) * (1.0 / s2b - 0.5) / 3.0  # bulk viscosity of rate s2b
        rows.append((xi - 2.0 * nu / 3.0, e))
        print(f"Poiseuille nu=0.1 non-slip: s2b={s2b:.4f} xi-2nu/3={xi - 2 * nu / 3:+.4f} E2={e:.3e}")
    ratios = [e / abs(d) for d, e in rows if abs(d) > 1e-12]
    smallest = min(rows, key=lambda r: r[1])
    assert abs(smallest[0]) < 1e-12 and smallest[1] < 1e-10
    assert max(ratios) / min(ratios) < 1.05  # E2 linear in |xi - 2 nu / 3|


# ----------------------------------------------------------------------------- Sec. III C: square duct
def test_duct_local_error_against_s3():
    a, F, nu = 16, 2e-4, 0.2
    n = 2 * a
    yc = np.arange(n) + 0.5 - a
    ua = analytic.duct_series(a, F, nu, yc, yc)  # [y, z]
    zs = (0.5, 7.5, 12.5)
    s3s = np.round(np.arange(1.20, 1.4201, 0.02), 4)
    E = np.zeros((len(s3s), 3))
    for i, s3 in enumerate(s3s):
        lat = _lattice((5, n, n), (0, 1, 1), "f64", workloads.rates(nu, s3=float(s3)), force=(F, 0.0, 0.0))
        lat.init()
        lat.step(8000)
        ux = _velocity(lat)[0].mean(axis=2)  # [z, y]
        lat.close()
        for j, z in enumerate(zs):
            k = int(z + a - 0.5)
            E[i, j] = np.sqrt(np.sum((ux[k] - ua[:, k]) ** 2) / np.sum(ua[:, k] ** 2))
        print(f"duct: s3={s3:.2f} E(0.5)={E[i, 0]:.3e} E(7.5)={E[i, 1]:.3e} E(12.5)={E[i, 2]:.3e}")
    best = [float(s3s[np.argmin(E[:, j])]) for j in range(3)]
    print(f"duct: s3 of smallest E(z) = {best} (paper: 1.33077 for z = 0.5 and 7.5, lower near the wall)")
    # the minima for z = 0.5 and 7.5 sit at the value the paper prints, 1.33077 (grid step 0.02)
    assert abs(best[0] - 1.33077) <= 0.02 and abs(best[1] - 1.33077) <= 0.02
    # near the wall (z = 12.5) the minimum moves away from it
    assert best[2] <= best[0] - 0.02
    assert E.min() < 5e-4


# ----------------------------------------------------------------------------- Sec. III D: forced TGV
def _forced_tgv_e2(L: int, storage: str, u0: float = 0.005, Re: float = 50.0):
    nu = u0 * L / Re
    k = 2.0 * np.pi / L
    T = int(round(4.0 * np.log(2.0) / (nu * 2.0 * k * k)))  # T* = 4
    ux, uy, Fx, Fy = analytic.forced_tgv_2d(L, u0, nu, 0.0)
    nz = 5
    u_init = np.zeros((3, nz, L, L))
    u_init[0] = ux[None]
    u_init[1] = uy[None]
    field = np.zeros((3, nz, L, L))
    field[0] = Fx[None]
    field[1] = Fy[None]
    lat = _lattice((L, L, nz), (0, 0, 0), storage, workloads.rates(nu), force_field=field)
    lat.init(np.ones((nz, L, L)), u_init)
    decay = 2.0 * nu * 2.0 * k * k  # force decays at twice the velocity rate
    for t in range(T):
        lat.set_force_scale(np.exp(-decay * t))  # F(t) at the collision of step t
        lat.step(1)
    lat.set_force_scale(np.exp(-decay * T))
    u = _velocity(lat)
    lat.close()
    ax, ay, _, _ = analytic.forced_tgv_2d(L, u0, nu, T)
    num = np.sum((u[0] - ax[None]) ** 2) + np.sum((u[1] - ay[None]) ** 2) + np.sum(u[2] ** 2)
    return float(np.sqrt(num / (nz * (np.sum(ax ** 2) + np.sum(ay ** 2))))), T


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_forced_taylor_green_second_order_convergence(storage):
    Ls = (16, 32, 64, 128)
    errs = []
    for L in Ls:
        e, T = _forced_tgv_e2(L, storage)
        errs.append(e)
        print(f"forced TGV {storage}: L={L} T={T} E2={e:.4e}")
    slope = np.polyfit(np.log(1.0 / np.array(Ls, float)), np.log(errs), 1)[0]  # E2 ~ dx^slope
    print(f"forced TGV {storage}: fitted slope {slope:.4f} (paper: 2.0345)")
    # FP32 storage adds its own error, about 5e-5 of u at L = 128 after 45 000 steps, which
    # moves the finest point by ~15%
    lo, hi = (1.95, 2.1) if storage == "f64" else (1.9, 2.2)
    assert lo < slope < hi
