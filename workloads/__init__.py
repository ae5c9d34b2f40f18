"""Seeded synthetic inputs for the D3Q27 cascaded LBM (arXiv:1801.04586).

This module only *generates inputs* -- initial density/velocity fields, force
fields, solid masks, relaxation-rate vectors and loss targets -- as float64 /
uint8 numpy arrays in the layouts both sides accept.  It holds none of the
method's arithmetic (no moments, equilibria, collision or streaming); the HIP
library and the CPU oracle each compute those themselves from these inputs.

Layouts: scalar fields (nz, ny, nx); vector fields (3, nz, ny, nx); masks
uint8 (nz, ny, nx) with 1 = solid.  Node (i, j, k) = (x, y, z).

Relaxation rates are the 10-vector (s0, s1, s2, s2b, s3, s3b, s4, s4b, s5, s6)
of Eq. (13), where the shear rate follows from the kinematic viscosity through
nu = (1/s2 - 1/2) c_s^2 (Sec. II B) and every other rate defaults to 1
(Sec. III).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Tuple

import numpy as np

SEED = 1801


def s2_from_nu(nu: float) -> float:
    """Shear rate for kinematic viscosity nu (lattice units, c_s^2 = 1/3)."""
    return 1.0 / (3.0 * nu + 0.5)


def rates(nu: float, s2b: Optional[float] = None, s3: float = 1.0, others: float = 1.0) -> np.ndarray:
    s2 = s2_from_nu(nu)
    r = np.full(10, float(others))
    r[2] = s2
    r[3] = float(others) if s2b is None else float(s2b)
    r[4] = float(s3)
    return r


def nonslip_s3(s2: float) -> float:
    """Rate s3 of the non-slip rule quoted in Sec. III B."""
    return (16.0 - 8.0 * s2) / (8.0 - s2)


def coords(n: int, walled: bool) -> np.ndarray:
    """Physical coordinate of node j: j + 1/2 on a walled axis (walls at 0 and n), j otherwise."""
    j = np.arange(n, dtype=np.float64)
    return j + 0.5 if walled else j


# --------------------------------------------------------------------------- configs
@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    dims: Tuple[int, int, int]          # (nx, ny, nz)
    walls: Tuple[int, int, int]
    nu: float
    steps: int
    storage: Tuple[str, ...]
    force_uniform: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    note: str = ""

    @property
    def n(self) -> int:
        return int(np.prod(self.dims))

    @property
    def shape(self):
        nx, ny, nz = self.dims
        return (nz, ny, nx)

    def rates(self) -> np.ndarray:
        return rates(self.nu)


POISEUILLE = Config("poiseuille_16x32x16", (16, 32, 16), (0, 1, 0), 0.1, 3000, ("f64",), (1e-6, 0.0, 0.0),
                    "force-driven channel, walls in y, gx = 1e-6, nu = 0.1, 3000 steps")
TGV128 = Config("taylor_green_128", (128, 128, 128), (0, 0, 0), 0.01, 1000, ("f64", "f32"), note="3D Taylor-Green, u0 = 0.04")
KOLMOGOROV512 = Config("kolmogorov_512", (512, 512, 512), (0, 0, 0), 0.005, 500, ("f64", "f32", "f16", "bf16"),
                       note="Kolmogorov forcing F0 sin(2 pi 4 y / Ny), F0 = 1e-5, perturbation 1e-3")
ADJOINT64 = Config("adjoint_channel_64", (64, 64, 64), (0, 1, 0), 0.05, 200, ("f32",),
                   note="learnable per-node force N(0, 1e-6^2), T = 200, checkpoint every 20")
POROUS = Config("porous_duct_640x320x320", (640, 320, 320), (0, 1, 1), 0.02, 2000, ("f32",), (2e-6, 0.0, 0.0),
                "random non-overlapping spheres r in [6, 12], solid fraction 0.2")


# --------------------------------------------------------------------------- fields
def taylor_green_3d(dims, u0: float = 0.04, with_pressure: bool = True):
    """3D Taylor-Green vortex on a 2 pi periodic box; node j -> 2 pi j / n.

    u = u0 (sin x cos y cos z, -cos x sin y cos z, 0).  With ``with_pressure``
    the initial density carries the incompressible pressure
    p = (u0^2/16)(cos 2x + cos 2y)(cos 2z + 2) as rho = 1 + p / c_s^2.
    Returns (rho (nz,ny,nx), u (3,nz,ny,nx)).
    """
    nx, ny, nz = dims
    x = 2.0 * np.pi * np.arange(nx) / nx
    y = 2.0 * np.pi * np.arange(ny) / ny
    z = 2.0 * np.pi * np.arange(nz) / nz
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    u = np.zeros((3, nz, ny, nx))
    u[0] = u0 * np.sin(X) * np.cos(Y) * np.cos(Z)
    u[1] = -u0 * np.cos(X) * np.sin(Y) * np.cos(Z)
    rho = np.ones((nz, ny, nx))
    if with_pressure:
        p = (u0 * u0 / 16.0) * (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0)
        rho = rho + 3.0 * p
    return rho, u


def kolmogorov_force(dims, F0: float = 1e-5, kf: int = 4) -> np.ndarray:
    """Per-node force field F_x = F0 sin(2 pi kf y / ny), other components 0."""
    nx, ny, nz = dims
    F = np.zeros((3, nz, ny, nx))
    prof = F0 * np.sin(2.0 * np.pi * kf * np.arange(ny) / ny)
    F[0] = prof[None, :, None]
    return F


def uniform_random_velocity(dims, amp: float = 1e-3, seed: int = SEED) -> np.ndarray:
    """i.i.d. U(-amp, amp) per component per node, (3, nz, ny, nx)."""
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, size=(3, nz, ny, nx))


def gaussian_force(dims, sigma: float = 1e-6, seed: int = SEED) -> np.ndarray:
    """i.i.d. N(0, sigma^2) per component per node, (3, nz, ny, nx)."""
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, sigma, size=(3, nz, ny, nx))


def channel_target(dims, walls, U: float = 1e-4) -> np.ndarray:
    """Target u_t = (U 4 y (H - y) / H^2, 0, 0) with y = j + 1/2 across a channel walled in y."""
    nx, ny, nz = dims
    y = coords(ny, bool(walls[1]))
    prof = U * 4.0 * y * (ny - y) / (ny * ny)
    ut = np.zeros((3, nz, ny, nx))
    ut[0] = prof[None, :, None]
    return ut


def random_state_fields(dims, seed: int, du: float = 0.05, drho: float = 0.02):
    """Random smooth-free (i.i.d.) density and velocity fields for parity tests."""
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    rho = 1.0 + rng.uniform(-drho, drho, size=(nz, ny, nx))
    u = rng.uniform(-du, du, size=(3, nz, ny, nx))
    return rho, u


def random_populations_perturbation(dims, seed: int, amp: float = 1e-3) -> np.ndarray:
    """i.i.d. U(-amp, amp) perturbation per population per node, (27, nz, ny, nx).

    Added to an equilibrium state, it excites every non-equilibrium moment."""
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, size=(27, nz, ny, nx))


def random_solids(dims, fraction: float, seed: int) -> np.ndarray:
    """i.i.d. Bernoulli(fraction) solid mask (uint8)."""
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    return (rng.random((nz, ny, nx)) < fraction).astype(np.uint8)


def porous_spheres(dims, walls=(0, 1, 1), rmin: float = 6.0, rmax: float = 12.0, solid_fraction: float = 0.2,
                   seed: int = SEED, max_tries: int = 2_000_000):
    """Random sequential addition of non-overlapping spheres.

    Centres are uniform in the box, radii U[rmin, rmax]; a candidate is kept
    when its distance to every kept centre is at least the sum of radii
    (distances periodic along periodic axes).  Spheres are clipped by walls
    and wrapped on periodic axes.  Stops when the solid node fraction reaches
    ``solid_fraction``.  Returns (mask uint8 (nz,ny,nx), centres (k,3), radii (k,)).
    """
    nx, ny, nz = dims
    L = np.array([nx, ny, nz], dtype=np.float64)
    per = np.array([not walls[0], not walls[1], not walls[2]])
    rng = np.random.default_rng(seed)
    mask = np.zeros((nz, ny, nx), dtype=np.uint8)
    n_total = nx * ny * nz
    n_solid = 0
    centres = np.zeros((0, 3))
    radii = np.zeros(0)
    tries = 0
    while n_solid < solid_fraction * n_total and tries < max_tries:
        tries += 1
        c = rng.uniform(0.0, 1.0, size=3) * L
        r = rng.uniform(rmin, rmax)
        if len(radii):
            d = centres - c
            d = np.where(per, d - L * np.round(d / L), d)
            if np.any(np.sum(d * d, axis=1) < (radii + r) ** 2):
                continue
        centres = np.vstack([centres, c])
        radii = np.append(radii, r)
        # rasterise: node (i, j, k) sits at coordinate (i, j, k) + 1/2 on walled axes, (i, j, k) otherwise
        off = np.where(per, 0.0, 0.5)
        lo = np.floor(c - r - off).astype(int)
        hi = np.ceil(c + r - off).astype(int)
        axes = []
        for a in range(3):
            idx = np.arange(lo[a], hi[a] + 1)
            pos = idx + off[a]
            if per[a]:
                idx_w = np.mod(idx, int(L[a]))
            else:
                keep = (idx >= 0) & (idx < int(L[a]))
                idx, pos = idx[keep], pos[keep]
                idx_w = idx
            axes.append((idx_w, pos))
        (ix, px), (iy, py), (iz, pz) = axes
        d2 = ((pz[:, None, None] - c[2]) ** 2 + (py[None, :, None] - c[1]) ** 2 + (px[None, None, :] - c[0]) ** 2)
        inside = d2 <= r * r
        sub = mask[np.ix_(iz, iy, ix)]
        add = inside & (sub == 0)
        n_solid += int(add.sum())
        mask[np.ix_(iz, iy, ix)] = np.where(inside, 1, sub).astype(np.uint8)
    return mask, centres, radii


def crop(a: np.ndarray, dims) -> np.ndarray:
    """Leading-corner crop of a (…, nz, ny, nx) array to dims (nx, ny, nz)."""
    nx, ny, nz = dims
    return np.ascontiguousarray(a[..., :nz, :ny, :nx])
