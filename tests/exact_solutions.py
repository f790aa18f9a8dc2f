"""Closed-form spacetimes used to pin the oracle (test-only).

Derivatives are taken with second-order forward-mode Taylor jets (value,
gradient, Hessian carried through numpy arithmetic), so every quantity below
is exact to rounding and none of it reuses the oracle's BSSN formulas:

  * Kerr in Kerr-Schild form: stationary, so every non-gauge BSSN right-hand
    side vanishes in the continuum; lapse and shift are those of the
    Kerr-Schild slicing;
  * Brill-Lindquist at t = 0 with alpha = psi^-2: d_t K_ij from the ADM
    evolution equation with K_ij = 0, i.e. -D_i D_j alpha + alpha R_ij, with
    the 3-Ricci tensor built from the Christoffel symbols of psi^4 delta;
  * the Kasner solution of the paper's cosmology example.

ADM data become BSSN slots through the paper's definitions:
phi = ln(det gamma)/12, gt = e^{-4 phi} gamma, K = gamma^ij K_ij,
At = e^{-4 phi}(K_ij - gamma_ij K / 3), Gt^i = gt^jk Gt^i_jk.
"""
import math

import numpy as np

SYM = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]


class Jet:
    """Truncated Taylor jet of a scalar field: value v, gradient g[3],
    Hessian H[3][3] (H may be None for first-order jets, g None for plain
    values)."""

    __slots__ = ("v", "g", "H")

    def __init__(self, v, g=None, H=None):
        self.v = np.asarray(v, dtype=float)
        self.g = g
        self.H = H

    @property
    def order(self):
        return 0 if self.g is None else (1 if self.H is None else 2)

    @staticmethod
    def lift(x):
        return x if isinstance(x, Jet) else Jet(x)

    def _trunc(self, o):
        return Jet(self.v, self.g if o >= 1 else None,
                   self.H if o >= 2 else None)

    def __add__(self, o):
        o = Jet.lift(o)
        if o.g is None:
            return Jet(self.v + o.v, self.g, self.H)
        if self.g is None:
            return Jet(self.v + o.v, o.g, o.H)
        n = min(self.order, o.order)
        return Jet(self.v + o.v, self.g + o.g,
                   self.H + o.H if n >= 2 else None)

    __radd__ = __add__

    def __neg__(self):
        return Jet(-self.v, None if self.g is None else -self.g,
                   None if self.H is None else -self.H)

    def __sub__(self, o):
        return self + (-Jet.lift(o))

    def __rsub__(self, o):
        return Jet.lift(o) + (-self)

    def __mul__(self, o):
        o = Jet.lift(o)
        if o.g is None:
            return Jet(self.v * o.v,
                       None if self.g is None else self.g * o.v,
                       None if self.H is None else self.H * o.v)
        if self.g is None:
            return o * self
        n = min(self.order, o.order)
        g = self.g * o.v + self.v * o.g
        H = None
        if n >= 2:
            H = (self.H * o.v + o.H * self.v
                 + np.einsum("i...,j...->ij...", self.g, o.g)
                 + np.einsum("i...,j...->ij...", o.g, self.g))
        return Jet(self.v * o.v, g, H)

    __rmul__ = __mul__

    def apply(self, f0, f1, f2):
        """Chain rule for a scalar function with derivatives f1, f2."""
        v = f0(self.v)
        if self.g is None:
            return Jet(v)
        d1 = f1(self.v)
        g = d1 * self.g
        H = None
        if self.H is not None:
            H = d1 * self.H + f2(self.v) * np.einsum("i...,j...->ij...",
                                                     self.g, self.g)
        return Jet(v, g, H)

    def recip(self):
        return self.apply(lambda x: 1 / x, lambda x: -1 / x**2,
                          lambda x: 2 / x**3)

    def __truediv__(self, o):
        o = Jet.lift(o)
        return self * o.recip()

    def __rtruediv__(self, o):
        return Jet.lift(o) * self.recip()

    def __pow__(self, p):
        return self.apply(lambda x: x**p, lambda x: p * x**(p - 1),
                          lambda x: p * (p - 1) * x**(p - 2))

    def sqrt(self):
        return self ** 0.5

    def log(self):
        return self.apply(np.log, lambda x: 1 / x, lambda x: -1 / x**2)

    def exp(self):
        return self.apply(np.exp, np.exp, np.exp)

    def d(self, k):
        """Partial derivative along axis k (one order lower)."""
        return Jet(self.g[k], None if self.H is None else self.H[k], None)


def coords(x, y, z, order=2):
    """Coordinate jets at arrays of points."""
    x, y, z = np.broadcast_arrays(np.asarray(x, float), np.asarray(y, float),
                                  np.asarray(z, float))
    out = []
    for k, c in enumerate((x, y, z)):
        g = np.zeros((3,) + c.shape)
        g[k] = 1.0
        H = np.zeros((3, 3) + c.shape) if order >= 2 else None
        out.append(Jet(c.copy(), g, H))
    return out


def det3(m):
    return (m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1])
            - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
            + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]))


def inv3(m):
    """Inverse by Cramer's rule (cofactors)."""
    d = det3(m)
    out = [[None] * 3 for _ in range(3)]
    for i in range(3):
        for j in range(3):
            r0, r1, c0, c1 = (j + 1) % 3, (j + 2) % 3, (i + 1) % 3, (i + 2) % 3
            out[i][j] = (m[r0][c0] * m[r1][c1] - m[r0][c1] * m[r1][c0]) / d
    return out


def _val(j):
    return j.v if isinstance(j, Jet) else np.asarray(j, float)


def adm_to_bssn(gam, K, alpha, beta):
    """25 BSSN slot arrays from ADM data; gam needs first derivatives (for
    Gt^i), K, alpha, beta values only."""
    det = det3(gam)
    phi = det.log() * (1.0 / 12.0)
    e4 = (phi * -4.0).exp()
    gt = [[gam[i][j] * e4 for j in range(3)] for i in range(3)]
    gamu = inv3([[Jet(_val(gam[i][j])) for j in range(3)] for i in range(3)])
    trK = sum(_val(gamu[i][j]) * _val(K[i][j]) for i in range(3)
              for j in range(3))
    e4v = _val(e4)
    At = [[(_val(K[i][j]) - _val(gam[i][j]) * trK / 3.0) * e4v
           for j in range(3)] for i in range(3)]
    gtu = inv3([[Jet(_val(gt[i][j])) for j in range(3)] for i in range(3)])
    gtu = [[_val(gtu[i][j]) for j in range(3)] for i in range(3)]
    dgt = [[[gt[i][j].g[k] for k in range(3)] for j in range(3)]
           for i in range(3)]
    # Christoffel symbols of the conformal metric, then Gt^i = g^jk G^i_jk
    Gam = []
    for i in range(3):
        s = 0.0
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    Gl = 0.5 * (dgt[l][j][k] + dgt[l][k][j] - dgt[j][k][l])
                    s = s + gtu[j][k] * gtu[i][l] * Gl
        Gam.append(s)
    slots = [_val(phi)] + [_val(gt[i][j]) for i, j in SYM] + [trK] + \
        [At[i][j] for i, j in SYM] + Gam + [_val(alpha)] + \
        [_val(b) for b in beta]
    shape = np.shape(slots[0])
    slots = [np.broadcast_to(np.asarray(s, float), shape) for s in slots]
    slots += [np.zeros(shape)] * 4
    return np.array(slots), trK


def kerr_schild(x, y, z, M=1.0, a=0.6):
    """Kerr in Kerr-Schild coordinates at arrays of points.  Returns
    (slots[25,...], ref) where ref holds the continuum right-hand sides of
    the gauge slots for 1+log slicing and a Gamma-driver with B = 0:
      ref['alpha'] = -2 alpha K + beta^j d_j alpha
      ref['beta']  = beta^j d_j beta^i           (3 components)
    Every other slot except B has continuum right-hand side zero."""
    X, Y, Z = coords(x, y, z, order=2)
    rho2 = X * X + Y * Y + Z * Z
    w = rho2 - a * a
    r2 = w * 0.5 + (w * w * 0.25 + Z * Z * (a * a)).sqrt()
    r = r2.sqrt()
    H = M * r2 * r / (r2 * r2 + Z * Z * (a * a))
    den = r2 + a * a
    l = [(r * X + Y * a) / den, (r * Y - X * a) / den, Z / r]
    gam = [[(H * 2.0) * l[i] * l[j] + (1.0 if i == j else 0.0)
            for j in range(3)] for i in range(3)]
    beta_low = [H * 2.0 * l[i] for i in range(3)]
    alpha = (H * 2.0 + 1.0) ** -0.5
    gamu = inv3(gam)
    beta = [sum((gamu[i][j] * beta_low[j] for j in range(3)), Jet(0.0))
            for i in range(3)]
    beta = [b if b.g is not None else b for b in beta]
    # stationary slices: K_ij = (L_beta gamma)_ij / (2 alpha)
    av = _val(alpha)
    K = [[None] * 3 for _ in range(3)]
    for i in range(3):
        for j in range(3):
            s = 0.0
            for k in range(3):
                s = s + _val(beta[k]) * gam[i][j].g[k]
                s = s + _val(gam[k][j]) * beta[k].g[i]
                s = s + _val(gam[i][k]) * beta[k].g[j]
            K[i][j] = s / (2.0 * av)
    slots, trK = adm_to_bssn(gam, K, alpha, beta)
    ref = {"alpha": -2.0 * av * trK + sum(_val(beta[k]) * alpha.g[k]
                                          for k in range(3)),
           "beta": np.array([sum(_val(beta[k]) * beta[i].g[k]
                                 for k in range(3)) for i in range(3)])}
    return slots, ref


def brill_lindquist_dtK(x, y, z, masses, centres):
    """Brill-Lindquist at t = 0, alpha = psi^-2, zero shift, K_ij = 0.
    Returns (d_t K, d_t At_ij for the 6 components) from
    d_t K_ij = -D_i D_j alpha + alpha R_ij and d_t At = e^{-4phi}[d_t K_ij]^TF
    (d_t phi = 0 at t = 0)."""
    X, Y, Z = coords(x, y, z, order=2)
    psi = Jet(1.0) + 0.0 * X
    for m, c in zip(masses, centres):
        r = ((X - c[0]) * (X - c[0]) + (Y - c[1]) * (Y - c[1])
             + (Z - c[2]) * (Z - c[2])).sqrt()
        psi = psi + m / (r * 2.0)
    p4 = psi ** 4
    alpha = psi ** -2
    # gamma = psi^4 delta; Christoffels (first-order jets) of gamma
    g = [[p4 if i == j else None for j in range(3)] for i in range(3)]

    def dg(i, j, k):  # d_k gamma_ij
        return p4.d(k) if i == j else None

    p4v = Jet(p4.v, p4.g, None)
    ginv = 1.0 / p4v  # first-order jet of 1/psi^4
    G2 = [[[None] * 3 for _ in range(3)] for _ in range(3)]
    for k in range(3):
        for i in range(3):
            for j in range(3):
                s = Jet(0.0)
                l = k  # gamma^kl diagonal
                for (aa, bb, cc, sg) in ((l, i, j, 1.0), (l, j, i, 1.0),
                                         (i, j, l, -1.0)):
                    t = dg(aa, bb, cc)
                    if t is not None:
                        s = s + t * sg
                G2[k][i][j] = ginv * s * 0.5 if s.g is not None else None
    R = np.zeros((3, 3) + np.shape(X.v))
    for i in range(3):
        for j in range(3):
            s = 0.0
            for k in range(3):
                if G2[k][i][j] is not None:
                    s = s + G2[k][i][j].g[k]
                if G2[k][i][k] is not None:
                    s = s - G2[k][i][k].g[j]
                for l in range(3):
                    if G2[k][k][l] is not None and G2[l][i][j] is not None:
                        s = s + G2[k][k][l].v * G2[l][i][j].v
                    if G2[k][j][l] is not None and G2[l][i][k] is not None:
                        s = s - G2[k][j][l].v * G2[l][i][k].v
            R[i, j] = s
    dtK = np.zeros_like(R)
    for i in range(3):
        for j in range(3):
            s = alpha.H[i, j].copy()
            for k in range(3):
                if G2[k][i][j] is not None:
                    s -= G2[k][i][j].v * alpha.g[k]
            dtK[i, j] = -s + alpha.v * R[i, j]
    gu = 1.0 / p4.v
    tr = gu * (dtK[0, 0] + dtK[1, 1] + dtK[2, 2])
    e4 = 1.0 / p4.v
    dtA = [(dtK[i, j] - (p4.v if i == j else 0.0) * tr / 3.0) * e4
           for i, j in SYM]
    return np.array([tr] + dtA)


def kasner_bssn(t):
    """Kasner: gamma = diag(t^4/3, t^4/3, t^-2/3), alpha = 1, beta = 0,
    K_ij = -d_t gamma_ij / 2 (= diag(-2/3 t^1/3, -2/3 t^1/3, 1/3 t^-5/3)),
    converted to the 25 BSSN slots by the definitions."""
    def slots_at(tt):
        g = [tt ** (4 / 3), tt ** (4 / 3), tt ** (-2 / 3)]
        k = [-(2 / 3) * tt ** (1 / 3), -(2 / 3) * tt ** (1 / 3),
             (1 / 3) * tt ** (-5 / 3)]
        det = g[0] * g[1] * g[2]
        phi = math.log(det) / 12
        e4 = math.exp(-4 * phi)
        trK = sum(k[i] / g[i] for i in range(3))
        At = [(k[i] - g[i] * trK / 3) * e4 for i in range(3)]
        gt = [g[i] * e4 for i in range(3)]
        out = np.zeros(25)
        out[0] = phi
        out[1], out[4], out[6] = gt
        out[7] = trK
        out[8], out[11], out[13] = At
        out[17] = 1.0
        return out
    return slots_at(t)


def kasner_dt(t):
    """d/dt of the Kasner BSSN slots, by hand-derived closed forms:
    phi = ln(t)/6, gt = diag(t^2/3, t^2/3, t^-4/3), K = -1/t,
    At = diag(-t^-1/3/3, -t^-1/3/3, 2 t^-7/3/3)."""
    out = np.zeros(25)
    out[0] = 1 / (6 * t)
    out[1] = out[4] = (2 / 3) * t ** (-1 / 3)
    out[6] = (-4 / 3) * t ** (-7 / 3)
    out[7] = 1 / t**2
    out[8] = out[11] = (1 / 9) * t ** (-4 / 3)
    out[13] = (-14 / 9) * t ** (-10 / 3)
    return out
