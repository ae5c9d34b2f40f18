"""Closed-form flows the paper verifies against (Sec. III), in lattice units.

These are independent of both the oracle and the HIP path: they are the exact
Navier-Stokes solutions quoted in the paper (or textbook results for the
same problems) and serve as pins for both.
"""
from __future__ import annotations

import numpy as np


def e2(u, ua) -> float:
    """Global relative error E2 = sqrt(sum |u - ua|^2 / sum |ua|^2) over all nodes (Sec. III B)."""
    u = np.asarray(u, dtype=np.float64)
    ua = np.asarray(ua, dtype=np.float64)
    return float(np.sqrt(np.sum((u - ua) ** 2) / np.sum(ua ** 2)))


def poiseuille_steady(H: int, F: float, nu: float) -> np.ndarray:
    """Steady Poiseuille profile (Sec. III B): u_x = F y (H - y) / (2 nu), y = j + 1/2, walls at 0, H."""
    y = np.arange(H) + 0.5
    return F * y * (H - y) / (2.0 * nu)


def poiseuille_startup(H: int, F: float, nu: float, t: float, nterms: int = 4001) -> np.ndarray:
    """Start-up of the same channel flow from rest (Fourier sine series of the diffusion problem)."""
    y = np.arange(H) + 0.5
    u = np.zeros(H)
    for n in range(1, nterms + 1, 2):
        k = n * np.pi / H
        u += 4.0 * F * H * H / (nu * np.pi ** 3 * n ** 3) * (1.0 - np.exp(-nu * k * k * t)) * np.sin(k * y)
    return u


def duct_series(a: float, F: float, nu: float, y, z, rho: float = 1.0, nterms: int = 401) -> np.ndarray:
    """Steady square-duct flow of Sec. III C, -a <= y, z <= a."""
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    Y, Z = np.meshgrid(y, z, indexing="ij")
    u = np.zeros_like(Y)
    for n in range(1, nterms + 1, 2):
        u += ((-1.0) ** ((n - 1) // 2) * (1.0 - np.cosh(n * np.pi * Z / (2 * a)) / np.cosh(n * np.pi / 2))
              * np.cos(n * np.pi * Y / (2 * a)) / n ** 3)
    return 16.0 * a * a * F / (rho * nu * np.pi ** 3) * u


def forced_tgv_2d(L: int, u0: float, nu: float, t: float):
    """Forced 2D Taylor-Green vortex (Sec. III D) on 0 <= x, y < 2 pi covered by L x L nodes.

    Returns (ux, uy) of shape (L, L) indexed [y, x] and the force field (Fx, Fy) at time t."""
    k = 2.0 * np.pi / L
    j = np.arange(L)
    Y, X = np.meshgrid(j * 1.0, j * 1.0, indexing="ij")
    x, y = k * X, k * Y  # physical angle 2 pi j / L, wave number 1 in angle units
    decay = np.exp(-nu * 2 * k * k * t)
    ux = -u0 * np.cos(x) * np.sin(y) * decay
    uy = u0 * np.sin(x) * np.cos(y) * decay
    fdec = np.exp(-2.0 * nu * 2 * k * k * t)
    Fx = -(k * u0 * u0 / 2.0) * np.sin(2 * x) * fdec
    Fy = -(k * u0 * u0 / 2.0) * np.sin(2 * y) * fdec
    return ux, uy, Fx, Fy


def kolmogorov_spinup(ny: int, F0: float, nu: float, t: float, kf: int = 4) -> np.ndarray:
    """Linear spin-up from rest under F_x = F0 sin(k y): u_x = F0/(nu k^2) (1 - exp(-nu k^2 t)) sin(k y)."""
    k = 2.0 * np.pi * kf / ny
    y = np.arange(ny)
    return F0 / (nu * k * k) * (1.0 - np.exp(-nu * k * k * t)) * np.sin(k * y)


def shear_wave(ny: int, A: float, B: float, nu: float, t: float) -> np.ndarray:
    """Decaying shear wave of Sec. III A: u_x = A sin(phi (y - B t)) exp(-phi^2 nu t), phi = 2 pi / ny."""
    phi = 2.0 * np.pi / ny
    y = np.arange(ny)
    return A * np.sin(phi * (y - B * t)) * np.exp(-phi * phi * nu * t)


def tgv3d_kinetic_energy_rate(nu: float, n: int) -> float:
    """Initial decay rate of the 3D Taylor-Green kinetic energy, KE'(0)/KE(0) = -6 nu k^2, k = 2 pi / n."""
    k = 2.0 * np.pi / n
    return -6.0 * nu * k * k
