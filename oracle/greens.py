"""Free-space 2-D Green's function and the area-included matrix G0 (FP64).

The paper starts every optimisation from a reference structure whose Green's
function is known analytically; its demonstration uses vacuum (Sec. IV, and the
remark in Sec. II that analytic initial Green's functions exist for simple
backgrounds).  In the 2-D TM reduction used here the scalar kernel solves
(lap + k0^2) g = -delta with outgoing waves under exp(-i w t):

    g(r) = (i/4) H0^(1)(k0 r).

Discretising Dyson's equation (eq. form2) with pixels of area h^2 turns the
integral into a sum whose weight b = k0^2 * deps * dV (eq. form4) we split as
alpha = k0^2 * deps times an area-included matrix:

    G0[p, q] = h^2 g(|r_p - r_q|)                    p != q (point sampled)
    G0[q, q] = integral of g over the disk of area h^2 (radius a = h/sqrt(pi))
             = (i pi a / (2 k0)) H1^(1)(k0 a) - 1/k0^2.

Pins (tests/test_oracle_greens.py): the small- and large-argument expansions of
H0, the source normalisation -ln(r)/(2 pi), the Helmholtz ODE away from the
source, and the self term against adaptive quadrature of g over the disk.
"""
from __future__ import annotations

import numpy as np
from scipy import special


def k0_of(problem) -> float:
    return 2.0 * np.pi / problem.wavelength


def g2d(r, k0: float):
    """(i/4) H0^(1)(k0 r), elementwise, r > 0."""
    return 0.25j * special.hankel1(0, k0 * np.asarray(r, dtype=np.float64))


def self_term(h: float, k0: float) -> complex:
    """Integral of g over the equal-area disk of a square pixel of side h."""
    a = h / np.sqrt(np.pi)
    return complex(1j * np.pi * a / (2.0 * k0) * special.hankel1(1, k0 * a) - 1.0 / k0**2)


def pixel_xy(problem) -> np.ndarray:
    """(N, 2) pixel centres; grid centred on the origin, p = iy*nx + ix."""
    h = problem.pitch
    x = (np.arange(problem.nx) - (problem.nx - 1) / 2.0) * h
    y = (np.arange(problem.ny) - (problem.ny - 1) / 2.0) * h
    X, Y = np.meshgrid(x, y)  # shape (ny, nx), row-major => p = iy*nx + ix
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def all_xy(problem) -> np.ndarray:
    """(R, 2) coordinates of the matrix rows: design pixels, then monitors."""
    return np.concatenate([pixel_xy(problem), problem.monitor_xy()], axis=0)


def incident_field(problem, xy=None) -> np.ndarray:
    """Unit plane wave exp(i k0 y) travelling +y (towards the monitors)."""
    if xy is None:
        xy = all_xy(problem)
    return np.exp(1j * k0_of(problem) * xy[:, 1])


def G0_block(problem, rows, cols) -> np.ndarray:
    """G0[rows, cols] (rows index design pixels then monitors, cols design pixels)."""
    k0 = k0_of(problem)
    h = problem.pitch
    N = problem.n
    xy = all_xy(problem)
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    d = xy[rows][:, None, :] - xy[cols][None, :, :]
    r = np.hypot(d[..., 0], d[..., 1])
    same = (rows[:, None] == cols[None, :]) & (rows[:, None] < N)
    r_safe = np.where(same, 1.0, r)
    out = h * h * g2d(r_safe, k0)
    out[same] = self_term(h, k0)
    return out


def build_G0(problem) -> np.ndarray:
    """Dense (R x N) complex128 G0 of the vacuum reference structure."""
    return G0_block(problem, np.arange(problem.rows), np.arange(problem.n))


def alpha_of(problem, eps) -> np.ndarray:
    """Contrast k0^2 (eps - eps_bg) per pixel (the paper's b divided by dV)."""
    return k0_of(problem) ** 2 * (np.asarray(eps, dtype=np.float64) - 1.0)
