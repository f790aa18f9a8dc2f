"""Pins of the multipole oracle (oracle/multipole.py) on the CPU:
  * for s = 0 Goldberg's sum is the ordinary spherical harmonic (scipy's,
    with the Condon-Shortley phase), l <= 6;
  * the textbook closed forms of -2Y_{2,+-2} and -2Y_{2,0};
  * the -2Y_lm, l <= 4, are orthonormal under the sphere quadrature (exact
    for Gauss-Legendre in cos(theta) with enough nodes);
  * the quadrature nodes and weights integrate cos^k(theta) exactly;
  * projections of grid functions that are polynomials of degree <= 3 per
    axis (interpolated exactly): z gives C^{10} = r^3 sqrt(4 pi / 3) and
    x + i y gives C^{11} = -r^3 sqrt(8 pi / 3), every other coefficient 0;
  * a sphere that reaches beyond the storage grid still interpolates a
    cubic exactly (clamped block).
"""
import math

import numpy as np
import pytest

from oracle import multipole as MP
from paper_1111_3344_amd import inputs as I

scipy_special = pytest.importorskip("scipy.special")


def _ylm_scipy(l, m, theta, phi):
    if hasattr(scipy_special, "sph_harm_y"):
        return scipy_special.sph_harm_y(l, m, theta, phi)
    return scipy_special.sph_harm(m, l, phi, theta)


def test_spin_zero_is_the_ordinary_harmonic():
    rng = np.random.default_rng(1)
    th = rng.uniform(0.05, math.pi - 0.05, 40)
    ph = rng.uniform(0, 2 * math.pi, 40)
    for l in range(7):
        for m in range(-l, l + 1):
            assert np.allclose(MP.swsh(0, l, m, th, ph),
                               _ylm_scipy(l, m, th, ph), rtol=1e-12,
                               atol=1e-13), (l, m)


def test_spin_minus_two_closed_forms():
    th = np.linspace(0.1, 3.0, 13)
    ph = np.linspace(0.0, 6.0, 13)
    c = math.sqrt(5 / (64 * math.pi))
    assert np.allclose(MP.swsh(-2, 2, 2, th, ph),
                       c * (1 + np.cos(th)) ** 2 * np.exp(2j * ph),
                       rtol=1e-13, atol=1e-14)
    assert np.allclose(MP.swsh(-2, 2, -2, th, ph),
                       c * (1 - np.cos(th)) ** 2 * np.exp(-2j * ph),
                       rtol=1e-13, atol=1e-14)
    assert np.allclose(MP.swsh(-2, 2, 0, th, ph),
                       math.sqrt(15 / (32 * math.pi)) * np.sin(th) ** 2,
                       rtol=1e-13, atol=1e-14)
    assert np.all(MP.swsh(-2, 1, 0, th, ph) == 0)


def test_orthonormal_under_the_quadrature():
    T, P, W = MP.sphere(6, 10)
    idx = [(l, m) for l in range(2, 5) for m in range(-l, l + 1)]
    Y = {k: MP.swsh(-2, k[0], k[1], T, P) for k in idx}
    for a in idx:
        for b in idx:
            ip = np.sum(np.conj(Y[a]) * Y[b] * W)
            assert abs(ip - (1.0 if a == b else 0.0)) < 1e-13, (a, b, ip)


def test_quadrature_integrates_powers_of_cos_theta():
    T, P, W = MP.sphere(5, 7)
    for k in range(10):
        want = 4 * math.pi / (k + 1) if k % 2 == 0 else 0.0
        assert abs(np.sum(np.cos(T) ** k * W) - want) < 1e-13, k


def _grid():
    return I.GridSpec((16, 15, 17), 3, (0.25, 0.25, 0.25), (-2.0, -1.9, -2.1),
                      I.BC_STATIC)


def _field(g, fn):
    X, Y, Z = g.mesh()
    return fn(X, Y, Z)


def test_projection_of_polynomial_fields():
    g = _grid()
    c, r = (0.1, -0.05, 0.02), 1.3
    C = MP.multipole(g, _field(g, lambda X, Y, Z: Z - c[2]), None, c, r, 0,
                     3, 24, 48)
    want = np.zeros(16, complex)
    want[2] = r ** 3 * math.sqrt(4 * math.pi / 3)
    assert np.allclose(C, want, rtol=0, atol=1e-11), C
    C = MP.multipole(g, _field(g, lambda X, Y, Z: X - c[0]),
                     _field(g, lambda X, Y, Z: Y - c[1]), c, r, 0, 3, 24, 48)
    want = np.zeros(16, complex)
    want[3] = -r ** 3 * math.sqrt(8 * math.pi / 3)
    assert np.allclose(C, want, rtol=0, atol=1e-11), C


def test_sphere_beyond_the_grid_still_exact_for_a_cubic():
    g = _grid()
    c, r = (0.0, 0.0, 0.0), 2.6            # leaves the storage grid
    f = _field(g, lambda X, Y, Z: 1.0 + X * Y * Z - 0.3 * Z ** 3)
    T, P, _ = MP.sphere(6, 12)
    pts = np.stack([r * np.sin(T) * np.cos(P), r * np.sin(T) * np.sin(P),
                    r * np.cos(T)], axis=1)
    got = MP.interpolate(g, f, pts)
    x, y, z = pts.T
    assert np.allclose(got, 1.0 + x * y * z - 0.3 * z ** 3, rtol=1e-12,
                       atol=1e-11)
