"""Mie series of a homogeneous dielectric cylinder (2-D TM), FP64.

Physics check of the discretised model: a disk of pixels flipped to eps must
scatter like a cylinder of the same area.  With incidence exp(i k0 y) expanded
by the Jacobi-Anger identity, exp(i x cos t) = sum_n i^n J_n(x) exp(i n t),
t = phi - pi/2, and continuity of E_z and dE_z/dr at r = R (mu = 1):

    x = k0 R,  m = sqrt(eps)
    a_n = [m J_n(x) J_n'(m x) - J_n'(x) J_n(m x)] /
          [H_n'(x) J_n(m x) - m H_n(x) J_n'(m x)]
    E_s(r, phi) = sum_n i^n a_n H_n^(1)(k0 r) exp(i n (phi - pi/2)).

Pins: a_n -> 0 as eps -> 1, and energy conservation for a lossless cylinder,
|1 + 2 a_n|^2 = 1 (each partial wave is a pure phase), both in
tests/test_oracle_greens.py.
"""
from __future__ import annotations

import numpy as np
from scipy import special


def coefficients(eps: float, x: float, nmax: int) -> np.ndarray:
    """a_n for n = -nmax..nmax (a_{-n} = a_n)."""
    m = np.sqrt(eps)
    n = np.arange(-nmax, nmax + 1)
    Jx, dJx = special.jv(n, x), special.jvp(n, x)
    Jmx, dJmx = special.jv(n, m * x), special.jvp(n, m * x)
    Hx, dHx = special.hankel1(n, x), special.h1vp(n, x)
    return (m * Jx * dJmx - dJx * Jmx) / (dHx * Jmx - m * Hx * dJmx)


def scattered_field(eps: float, radius: float, k0: float, points, nmax: int = 30) -> np.ndarray:
    """Scattered E_z at points outside a cylinder centred on the origin."""
    pts = np.asarray(points, dtype=np.float64)
    r = np.hypot(pts[:, 0], pts[:, 1])
    phi = np.arctan2(pts[:, 1], pts[:, 0])
    a = coefficients(eps, k0 * radius, nmax)
    n = np.arange(-nmax, nmax + 1)
    terms = (1j ** n)[None, :] * a[None, :] * special.hankel1(n[None, :], k0 * r[:, None]) \
        * np.exp(1j * n[None, :] * (phi[:, None] - np.pi / 2))
    return terms.sum(axis=1)
