"""Multipole coefficients of a complex grid function on a coordinate sphere,
plain numpy in FP64.  Test infrastructure only.

It follows the paper's description of the multipole module (analysis
section, next to the Weyl scalar): the field u is interpolated onto a
coordinate sphere of radius r and projected onto spin-weighted spherical
harmonics,
    C^{lm}(r) = integral of conj(sY_lm) u r^2 dOmega.

Readings (the paper gives neither the harmonics' convention nor the
quadrature):
  * sY_lm is Goldberg's explicit sum (which for s = 0 is the ordinary
    harmonic with the Condon-Shortley phase):
      sY_lm = (-1)^m sqrt((l+m)!(l-m)!(2l+1) / (4 pi (l+s)!(l-s)!))
              sin^{2l}(theta/2) e^{i m phi}
              sum_r C(l-s, r) C(l+s, r+s-m) (-1)^{l-r-s} cot^{2r+s-m}(theta/2);
  * the sphere carries n_theta Gauss-Legendre nodes in cos(theta) and n_phi
    uniform points in phi (phi_k = 2 pi k / n_phi); the integral is the sum
    of f w_j (2 pi / n_phi) over them (w_j the Gauss-Legendre weights),
    which is exact for the products of harmonics of one spin (polynomials
    in cos(theta) times e^{i m phi}) up to the node counts; the factor r^2
    is kept as the paper writes it;
  * the point x = c + r (sin theta cos phi, sin theta sin phi, cos theta)
    takes the tricubic Lagrange interpolation of the field on the 4 x 4 x 4
    storage points around it (the rule of puncture tracking, oracle/adm.py).
"""
import math

import numpy as np

from . import adm as _adm


def swsh(s, l, m, theta, phi):
    """Goldberg's sY_lm at (theta, phi) (arrays), theta strictly inside
    (0, pi)."""
    if l < abs(s) or abs(m) > l:
        return np.zeros(np.broadcast(theta, phi).shape, complex)
    pre = (-1) ** m * math.sqrt(
        math.factorial(l + m) * math.factorial(l - m) * (2 * l + 1)
        / (4 * math.pi * math.factorial(l + s) * math.factorial(l - s)))
    half = np.asarray(theta) / 2.0
    cot = np.cos(half) / np.sin(half)
    total = 0.0
    for r in range(0, l - s + 1):
        k = r + s - m
        if k < 0 or k > l + s:
            continue
        total = total + (math.comb(l - s, r) * math.comb(l + s, k)
                         * (-1) ** (l - r - s) * cot ** (2 * r + s - m))
    return pre * np.sin(half) ** (2 * l) * total * np.exp(1j * m * phi)


def sphere(ntheta, nphi):
    """(theta, phi, weight) of every quadrature point, theta slowest (in the
    order of the Gauss-Legendre nodes, cos(theta) ascending)."""
    x, w = np.polynomial.legendre.leggauss(ntheta)
    th = np.arccos(x)
    ph = np.arange(nphi) * 2 * math.pi / nphi
    T, P = np.meshgrid(th, ph, indexing="ij")
    W = np.meshgrid(w, ph, indexing="ij")[0] * (2 * math.pi / nphi)
    return T.ravel(), P.ravel(), W.ravel()


def interpolate(grid, f, pts):
    """Tricubic interpolation of the storage-grid array f (z, y, x) at the
    points pts (n, 3)."""
    out = np.zeros(len(pts))
    for n, x in enumerate(np.asarray(pts, float)):
        base, wts = [], []
        for a in range(3):
            N = grid.n[a] + 2 * grid.ghost
            x0 = grid.origin[a] - grid.ghost * grid.h[a]
            s = (x[a] - x0) / grid.h[a]
            b = min(max(int(np.floor(s)) - 1, 0), N - 4)
            base.append(b)
            wts.append(_adm.lagrange4(s - b))
        acc = 0.0
        for k in range(4):
            for j in range(4):
                for i in range(4):
                    acc += (wts[2][k] * wts[1][j] * wts[0][i] *
                            f[base[2] + k, base[1] + j, base[0] + i])
        out[n] = acc
    return out


def multipole(grid, re, im, centre, radius, s, lmax, ntheta, nphi):
    """C^{lm} for l = 0..lmax, m = -l..l as a complex array indexed
    l*l + l + m (zero for l < |s|).  re, im: storage-grid arrays (z, y, x)
    of the field's real and imaginary parts (im may be None)."""
    T, P, W = sphere(ntheta, nphi)
    pts = np.stack([centre[0] + radius * np.sin(T) * np.cos(P),
                    centre[1] + radius * np.sin(T) * np.sin(P),
                    centre[2] + radius * np.cos(T)], axis=1)
    u = interpolate(grid, re, pts).astype(complex)
    if im is not None:
        u = u + 1j * interpolate(grid, im, pts)
    out = np.zeros((lmax + 1) ** 2, complex)
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            Y = swsh(s, l, m, T, P)
            out[l * l + l + m] = np.sum(np.conj(Y) * u * W) * radius ** 2
    return out
