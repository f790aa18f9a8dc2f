"""Pins of the ADM -> BSSN conversion oracle (oracle/adm.py) against what
the definitions fix, on the CPU:
  * identities of the converted state: det gt = 1, At traceless, and the
    ADM metric and extrinsic curvature rebuilt from it;
  * Brill-Lindquist data (g = psi^4 delta, K = 0): phi = ln psi, gt = delta,
    At = K = Gt = 0;
  * Gt^i = -d_j gt^ij for det gt = 1, with the exact derivative taken by
    complex-step differentiation of an analytic metric: the converted Gt
    converges to it at fourth order;
  * the cubic extrapolation of the ghost layers reproduces a cubic
    polynomial exactly (faces, edges, corners), and takes the edge normal
    (1, 1, 0) (a hand-computed value);
  * puncture tracking: the tricubic interpolation is exact for a shift
    that is a cubic in each coordinate (inside, near the edge, in the
    ghosts) and returns the node value at a node; a constant shift moves a
    puncture by exactly -beta dt.
"""
import numpy as np

from oracle import adm as A
from paper_1111_3344_amd import inputs as I


def _adm_smooth(g, seed=1):
    """Smooth positive-definite metric, smooth K_ij, lapse and shift."""
    rng = np.random.default_rng(seed)
    X, Y, Z = g.mesh()
    adm = np.zeros(g.off0 + 16 * g.sf)
    v = g.view(adm, 16)
    for s in range(16):
        k = rng.uniform(0.5, 1.5, 3)
        ph = rng.uniform(0, 2 * np.pi)
        w = np.sin(k[0] * X + k[1] * Y + k[2] * Z + ph)
        if s in (0, 3, 5):
            v[s] = 1.0 + 0.2 * w
        elif s < 6:
            v[s] = 0.05 * w
        elif s == 12:
            v[s] = 1.0 + 0.1 * w
        else:
            v[s] = 0.1 * w
    return adm


def _grid(n=10, h=0.15, ghost=3):
    return I.GridSpec((n, n + 1, n + 2), ghost, (h, 1.1 * h, 0.9 * h),
                      (-0.7, -0.4, -0.6), I.BC_STATIC)


def test_conversion_identities():
    g = _grid()
    adm = _adm_smooth(g)
    u = A.from_adm(g, adm)
    v = g.view(u)
    a = g.view(adm, 16)
    gt = A._mat(v[A.GXX:A.GXX + 6])
    assert np.allclose(A._det(gt), 1.0, rtol=0, atol=1e-14)
    gtu = A._inv(gt)
    tr = sum(gtu[i, j] * v[A.AXX + A.SYM[(i, j)]]
             for i in range(3) for j in range(3))
    assert np.abs(tr).max() < 1e-14
    e4 = np.exp(4 * v[A.PHI])
    for m in range(6):
        assert np.allclose(e4 * v[A.GXX + m], a[m], rtol=1e-14, atol=1e-15)
        assert np.allclose(e4 * (v[A.AXX + m] + v[A.GXX + m] * v[A.TRK] / 3),
                           a[6 + m], rtol=1e-13, atol=1e-15)
    assert np.array_equal(v[A.ALP], a[12])
    assert np.array_equal(v[A.BETX:A.BETX + 3], a[13:16])
    assert np.all(v[A.BX:A.BX + 3] == 0) and np.all(v[A.ADOT] == 0)


def test_brill_lindquist_conversion():
    g = I.cell_centred(16, 1.0, 3.0, 3)
    X, Y, Z = g.mesh()
    r = np.sqrt(X * X + Y * Y + Z * Z)
    psi = 1 + 0.5 / r
    adm = np.zeros(g.off0 + 16 * g.sf)
    v = g.view(adm, 16)
    for s in (0, 3, 5):
        v[s] = psi ** 4
    v[12] = psi ** -2
    u = g.view(A.from_adm(g, adm))
    assert np.allclose(u[A.PHI], np.log(psi), rtol=1e-14, atol=1e-15)
    for m in range(6):
        want = 1.0 if m in (0, 3, 5) else 0.0
        assert np.abs(u[A.GXX + m] - want).max() < 1e-14
        assert np.abs(u[A.AXX + m]).max() == 0
    assert np.abs(u[A.TRK]).max() == 0
    assert np.abs(u[A.GAMX:A.GAMX + 3]).max() < 1e-11


def _metric(X, Y, Z):
    """Analytic metric (accepts complex coordinates), (3, 3, ...)."""
    w = np.sin(0.9 * X + 0.4 * Y - 0.3 * Z)
    q = np.cos(0.5 * X - 0.7 * Y + 0.8 * Z)
    return np.array([[1 + 0.3 * w, 0.1 * q, 0.05 * w * q],
                     [0.1 * q, 1 + 0.2 * q, 0.07 * w],
                     [0.05 * w * q, 0.07 * w, 1 + 0.25 * w * q]])


def _exact_gamma(X, Y, Z, eps=1e-30):
    """Gt^i = -d_j gt^ij, gt^ij = (det g)^(1/3) g^ij, by complex steps."""
    out = np.zeros((3,) + X.shape)
    for j in range(3):
        d = [0, 0, 0]
        d[j] = 1j * eps
        gm = _metric(X + d[0], Y + d[1], Z + d[2])
        gtu = _det_c(gm) ** (1.0 / 3.0) * A._inv(gm)
        for i in range(3):
            out[i] -= np.imag(gtu[i, j]) / eps
    return out


def _det_c(m):
    return A._det(m)


def test_conformal_connection_fourth_order():
    errs = []
    for n in (12, 24):
        h = 1.2 / n
        g = I.GridSpec((n, n, n), 3, (h, h, h), (0.1, -0.2, 0.3),
                       I.BC_STATIC)
        X, Y, Z = g.mesh()
        adm = np.zeros(g.off0 + 16 * g.sf)
        v = g.view(adm, 16)
        gm = _metric(X, Y, Z)
        for (i, j), m in ((k, A.SYM[k]) for k in
                          [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]):
            v[m] = gm[i, j]
        u = g.view(A.from_adm(g, adm))
        gc = g.ghost
        got = u[A.GAMX:A.GAMX + 3, gc:-gc, gc:-gc, gc:-gc]
        ex = _exact_gamma(X, Y, Z)[:, gc:-gc, gc:-gc, gc:-gc]
        errs.append(np.abs(got - ex).max())
    ratio = errs[0] / errs[1]
    assert 12 < ratio < 20, (errs, ratio)


def test_cubic_extrapolation():
    g = I.GridSpec((7, 6, 8), 3, (0.1, 0.2, 0.15), (0.3, -0.4, 0.2),
                   I.BC_STATIC)
    X, Y, Z = g.mesh()
    P = (1.5 - 0.3 * X + 0.7 * Y * Z - 0.2 * X ** 3 + 0.4 * X * Y * Z
         + 0.1 * Z ** 2 * Y - 0.6 * Y ** 3)
    f = np.zeros((1,) + X.shape)
    gc = g.ghost
    f[0, gc:-gc, gc:-gc, gc:-gc] = P[gc:-gc, gc:-gc, gc:-gc]
    A.extrapolate_layers(g, f)
    assert np.allclose(f[0], P, rtol=1e-12, atol=1e-12)
    # arbitrary interior values: the (+x, +y) edge point of layer 1 takes
    # the diagonal stencil
    rng = np.random.default_rng(3)
    f = np.zeros((1,) + X.shape)
    f[0, gc:-gc, gc:-gc, gc:-gc] = rng.normal(size=(8, 6, 7))
    A.extrapolate_layers(g, f)
    ex, ey = 7 + gc, 6 + gc
    z = gc + 2
    vals = [f[0, z, ey - m, ex - m] for m in range(1, 5)]
    want = 4 * vals[0] - 6 * vals[1] + 4 * vals[2] - vals[3]
    assert f[0, z, ey, ex] == want


def _shift_grid():
    return I.GridSpec((9, 8, 10), 3, (0.2, 0.15, 0.25), (-0.9, -0.5, -1.1),
                      I.BC_STATIC)


def test_tracker_exact_for_tricubic_shift():
    g = _shift_grid()
    X, Y, Z = g.mesh()

    def beta(x, y, z):
        return np.array([0.3 - 0.2 * x ** 3 + 0.5 * x * y * z,
                         0.1 * y ** 2 * z - 0.4 * x * y ** 3,
                         -0.2 + 0.6 * x ** 2 * y * z ** 3])
    u = g.empty()
    v = g.view(u)
    b = beta(X, Y, Z)
    for c in range(3):
        v[A.BETX + c] = b[c]
    pos = np.array([[0.13, 0.21, -0.37], [-0.5, 0.02, 0.6],
                    [0.9, 0.6, 1.0],          # near the far edge
                    [-1.4, -0.9, -1.6]])      # in the ghost region
    dt = 0.05
    new = A.track_punctures(g, u, pos, dt)
    want = pos - dt * np.stack([beta(*p) for p in pos])
    assert np.allclose(new, want, rtol=1e-13, atol=1e-14)


def test_tracker_at_a_grid_point_and_constant_shift():
    g = _shift_grid()
    u = g.empty()
    v = g.view(u)
    rng = np.random.default_rng(9)
    v[A.BETX:A.BETX + 3] = rng.normal(size=v[A.BETX:A.BETX + 3].shape)
    # storage point (4, 5, 6): its own value exactly (weights 0, 1, 0, 0)
    x = [g.origin[a] + ((4, 5, 6)[a] - g.ghost) * g.h[a] for a in range(3)]
    b = A.shift_at(g, u, [x])[0]
    assert np.allclose(b, v[A.BETX:A.BETX + 3, 6, 5, 4], rtol=1e-14,
                       atol=1e-15)
    v[A.BETX:A.BETX + 3] = np.array([0.3, -0.2, 0.1]).reshape(3, 1, 1, 1)
    new = A.track_punctures(g, u, [[0.05, -0.07, 0.11]], 0.5)
    assert np.allclose(new, [[0.05 - 0.15, -0.07 + 0.1, 0.11 - 0.05]],
                       rtol=0, atol=1e-15)
