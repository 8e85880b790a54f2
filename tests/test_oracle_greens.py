"""Pins of the oracle's free-space kernel, self term, G0 and Mie series.

Each test checks the oracle against something other than itself: series
expansions of H0 (Abramowitz & Stegun 9.1.12-9.1.13 and Hankel's asymptotic
expansion 9.2.7), the Helmholtz ODE, the logarithmic source normalisation,
adaptive quadrature of the log-singular self integral, and exact properties
of the Mie coefficients.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import greens, mie, state
import workloads as W

EULER_GAMMA = 0.5772156649015329


def _h0_series(x):
    """H0^(1)(x) = J0 + i Y0 from the ascending series (A&S 9.1.12, 9.1.13)."""
    q = x * x / 4.0
    J0 = 0.0
    Ysum = 0.0
    term = 1.0
    harm = 0.0
    for k in range(0, 60):
        if k > 0:
            term *= -q / (k * k)
            harm += 1.0 / k
        J0 += term
        if k > 0:
            Ysum += -term * harm     # (-1)^(k+1) H_k q^k/(k!)^2 = -term*H_k
    Y0 = (2.0 / math.pi) * (math.log(x / 2.0) + EULER_GAMMA) * J0 + (2.0 / math.pi) * Ysum
    return complex(J0, Y0)


def _h0_asymptotic(x, terms=8):
    """Hankel's expansion H0^(1)(x) ~ sqrt(2/(pi x)) e^{i(x - pi/4)} sum_k i^k a_k x^-k."""
    s = 0j
    a = 1.0
    for k in range(terms):
        if k > 0:
            a *= -((2 * k - 1) ** 2) / (k * 8.0)
        s += (1j ** k) * a / x**k
    return math.sqrt(2.0 / (math.pi * x)) * np.exp(1j * (x - math.pi / 4)) * s


@pytest.mark.parametrize("x", [1e-3, 0.05, 0.3, 1.0, 2.5])
def test_kernel_small_argument_series(x):
    k0 = 2 * math.pi
    g = complex(greens.g2d(x / k0, k0))
    ref = 0.25j * _h0_series(x)
    assert abs(g - ref) <= 1e-12 * abs(ref)


@pytest.mark.parametrize("x", [40.0, 80.0, 200.0])
def test_kernel_large_argument_expansion(x):
    k0 = 2 * math.pi
    g = complex(greens.g2d(x / k0, k0))
    ref = 0.25j * _h0_asymptotic(x)
    assert abs(g - ref) <= 1e-9 * abs(ref)


def test_kernel_source_normalisation():
    """(lap + k0^2) g = -delta  <=>  g ~ -ln(r)/(2 pi) near the source, Im g(0) = 1/4."""
    k0 = 2 * math.pi
    r1, r2 = 1e-7, 3e-7
    g1, g2 = greens.g2d(r1, k0), greens.g2d(r2, k0)
    assert abs((g1.real - g2.real) - (-(math.log(r1 / r2)) / (2 * math.pi))) < 1e-10
    assert abs(g1.imag - 0.25) < 1e-10


def test_kernel_solves_helmholtz_away_from_source():
    """Radial ODE g'' + g'/r + k0^2 g = 0, and outgoing phase (Im part leads)."""
    k0 = 2 * math.pi / 1.3
    r, d = 0.7, 1e-3
    gm, g0, gp = greens.g2d([r - d, r, r + d], k0)
    lhs = (gp - 2 * g0 + gm) / d**2 + (gp - gm) / (2 * d * r) + k0**2 * g0
    assert abs(lhs) < 1e-5 * k0**2 * abs(g0)
    # outgoing wave exp(+i k0 r) under exp(-i w t): phase increases with r
    far = greens.g2d([50.0, 50.0 + 0.01], k0)
    dphase = np.angle(far[1] / far[0])
    assert abs(dphase - k0 * 0.01) < 1e-3


@pytest.mark.parametrize("h,wl", [(0.05, 1.0), (1 / 16, 1.0), (0.05, 0.8), (0.05, 1.2)])
def test_self_term_equals_disk_quadrature(h, wl):
    k0 = 2 * math.pi / wl
    a = h / math.sqrt(math.pi)
    re = integrate.quad(lambda r: 2 * math.pi * r * greens.g2d(r, k0).real, 0.0, a,
                        limit=200, epsabs=1e-16, epsrel=1e-13)[0]
    im = integrate.quad(lambda r: 2 * math.pi * r * greens.g2d(r, k0).imag, 0.0, a,
                        limit=200, epsabs=1e-16, epsrel=1e-13)[0]
    st = greens.self_term(h, k0)
    assert abs(st - complex(re, im)) <= 1e-10 * abs(st)


def test_G0_structure():
    p = W.tiny(5, 7, n_mon=4)
    G0 = greens.build_G0(p)
    N = p.n
    assert G0.shape == (p.rows, N)
    D = G0[:N]
    assert np.array_equal(D, D.T)                                    # reciprocity
    st = greens.self_term(p.pitch, greens.k0_of(p))
    assert np.allclose(np.diagonal(D), st, rtol=0, atol=0)
    # translation invariance: G0[(iy,ix),(jy,jx)] depends on (|iy-jy|, |ix-jx|) only
    a = D[0 * 7 + 1, 2 * 7 + 4]
    b = D[3 * 7 + 6, 1 * 7 + 3]
    assert a == b
    # off-diagonal = h^2 (i/4) H0(k0 r)
    r = math.hypot(2 * p.pitch, 3 * p.pitch)
    assert abs(a - p.pitch**2 * greens.g2d(r, greens.k0_of(p))) < 1e-18
    # monitors: all on one line beyond the grid, centre one on the axis
    mxy = p.monitor_xy()
    assert mxy[p.fom_monitor, 0] == 0.0
    assert np.all(mxy[:, 1] > p.ny * p.pitch / 2)


def test_incident_field_and_empty_structure_fom():
    p = W.SMALL_32
    E = greens.incident_field(p)
    assert np.allclose(np.abs(E), 1.0)
    _, E1 = state.dense_state(W.tiny(4, 4), np.ones(16))
    assert np.allclose(E1, greens.incident_field(W.tiny(4, 4)), atol=1e-15)


# ---------------------------------------------------------------------- Mie
def test_mie_lossless_partial_waves_are_phases():
    a = mie.coefficients(12.25, 2 * math.pi * 0.3, 12)
    assert np.allclose(np.abs(1 + 2 * a), 1.0, atol=1e-12)
    assert np.allclose(mie.coefficients(1.0, 1.7, 8), 0.0, atol=1e-15)


def _disk_problem(h, radius, wl=1.0):
    n = int(math.ceil(2 * radius / h)) + 2
    p = W.tiny(n, n, n_mon=2, pitch=h, wavelength=wl)
    xy = greens.pixel_xy(p)
    inside = np.hypot(xy[:, 0], xy[:, 1]) < radius
    return p, inside


def _mie_rel_error(eps, h, radius):
    p, inside = _disk_problem(h, radius)
    k0 = greens.k0_of(p)
    eps_arr = np.where(inside, eps, 1.0)
    R_eq = math.sqrt(inside.sum() * h * h / math.pi)
    phi = np.linspace(0, 2 * math.pi, 24, endpoint=False)
    pts = np.stack([1.5 * np.cos(phi), 1.5 * np.sin(phi)], axis=1)
    Es_d = state.field_at(p, eps_arr, pts) - np.exp(1j * k0 * pts[:, 1])
    Es_m = mie.scattered_field(eps, R_eq, k0, pts)
    return np.linalg.norm(Es_d - Es_m) / np.linalg.norm(Es_m)


def test_discrete_model_matches_mie_series():
    """A pixelated disk (eps 2.25, R = lambda/4) scatters like the cylinder of equal area."""
    e20 = _mie_rel_error(2.25, 1 / 20, 0.25)
    e40 = _mie_rel_error(2.25, 1 / 40, 0.25)
    assert e20 < 2e-2
    assert e40 < e20 / 2


@pytest.mark.slow
def test_discrete_model_converges_to_mie_high_contrast():
    e40 = _mie_rel_error(12.25, 1 / 40, 0.25)
    e80 = _mie_rel_error(12.25, 1 / 80, 0.25)
    assert e80 < e40 and e80 < 0.06
