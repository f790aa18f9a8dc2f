"""Pins of the Psi_4 oracle (oracle/psi4.py) on the CPU.

  * The 4-D reference (tests/spacetime4.py) is itself pinned: the
    Kretschmann scalar of Schwarzschild in Kerr-Schild coordinates is
    48 M^2 / r^6, and the Ricci tensor of both test space-times vanishes.
  * The fiducial triad: for the flat metric it is the textbook spherical
    basis (rhat = x/r, thetahat = (cos th cos ph, cos th sin ph, -sin th),
    phihat = (-sin ph, cos ph, 0)); for any metric it is orthonormal, phihat
    is along (-y, x, 0), rhat lies in the span of (-y, x, 0) and (x, y, z)
    with a positive (x, y, z) part, and thetahat points along the
    unnormalised theta vector of the definition.
  * psi4_point (the 3+1 projection formula with the Gauss, Codazzi and
    Ricci equations) equals R_abcd n^a mb^b n^c mb^d computed from the
    4-Riemann tensor of two exact vacuum space-times: a pp-wave with a
    time-dependent profile, and Schwarzschild in Kerr-Schild coordinates
    with the hole away from the tetrad's centre (the tetrad then does not
    follow the principal null directions and Psi_4 != 0).  With the hole
    at the tetrad's centre the tetrad's l and n lie along the principal
    null directions and Psi_4 = 0.
  * The grid function psi4: on cubic-polynomial BSSN data (every stencil
    exact) it equals psi4_point fed with exact derivatives, at order 4 and
    8; Minkowski gives exactly 0; flat space in curvilinear coordinates
    (quadratic coordinate map, so the metric is a polynomial the stencils
    differentiate exactly) gives 0 to rounding; on a discretised pp-wave
    slice the error falls 2^4 per halving of h at order 4.
"""
import math

import numpy as np
import pytest

from oracle import psi4 as P
from paper_1111_3344_amd import inputs as I

sympy = pytest.importorskip("sympy")
import spacetime4 as S4  # noqa: E402  (tests/ is on sys.path)


@pytest.fixture(scope="module")
def ppw():
    return S4.pp_wave()


@pytest.fixture(scope="module")
def schw_off():
    return S4.schwarzschild_ks(M=1, centre=(0.4, -0.3, 0.2))


def _triad_at(gam, x):
    rh, th, ph = P.tetrad(gam[:, :, None], np.asarray(x, float)[:, None])
    return rh[:, 0], th[:, 0], ph[:, 0]


def _psi4_3p1(st, p, centre=(0.0, 0.0, 0.0)):
    gam, dg, ddg, K, dK, _, _ = st.adm(p)
    x = np.asarray(p[1:]) - np.asarray(centre)
    e = lambda a: a[..., None]
    return P.psi4_point(e(gam), e(dg), e(ddg), e(K), e(dK), x[:, None])[0]


# ---- the 4-D reference ---------------------------------------------------------

def test_reference_kretschmann_and_ricci():
    st = S4.schwarzschild_ks(M=1)
    for p in [(0.0, 3.0, 1.0, -2.0), (0.7, -2.5, 2.0, 1.5)]:
        R = st.riemann_down(p)
        gi = np.linalg.inv(st.metric(p))
        Ru = np.einsum("ai,bj,ck,dl,ijkl->abcd", gi, gi, gi, gi, R)
        r = math.sqrt(sum(v * v for v in p[1:]))
        assert np.einsum("abcd,abcd->", R, Ru) == pytest.approx(
            48.0 / r**6, rel=1e-12)
        ric = np.einsum("ac,abcd->bd", gi, R)
        assert np.abs(ric).max() < 1e-14
    st = S4.pp_wave()
    for p in [(0.3, 0.5, -0.7, 0.2), (1.1, -0.4, 0.9, 0.6)]:
        R = st.riemann_down(p)
        gi = np.linalg.inv(st.metric(p))
        assert np.abs(R).max() > 0.05
        assert np.abs(np.einsum("ac,abcd->bd", gi, R)).max() < 1e-14


# ---- the triad ---------------------------------------------------------------------

def test_triad_flat_is_spherical_basis():
    rng = np.random.default_rng(5)
    x = rng.uniform(-2, 2, (3, 20))
    gam = np.broadcast_to(np.eye(3)[:, :, None], (3, 3, 20))
    rh, th, ph = P.tetrad(gam, x)
    r = np.linalg.norm(x, axis=0)
    rho = np.hypot(x[0], x[1])
    cth, sth = x[2] / r, rho / r
    cph, sph = x[0] / rho, x[1] / rho
    assert np.allclose(rh, x / r, atol=1e-14)
    assert np.allclose(th, [cth * cph, cth * sph, -sth], atol=1e-14)
    assert np.allclose(ph, [-sph, cph, 0 * cph], atol=1e-14)


def test_triad_defining_properties():
    rng = np.random.default_rng(6)
    npt = 30
    x = rng.uniform(-2, 2, (3, npt))
    A = rng.uniform(-0.3, 0.3, (3, 3, npt))
    gam = np.einsum("ki...,kj...->ij...", A + np.eye(3)[:, :, None],
                    A + np.eye(3)[:, :, None])
    rh, th, ph = P.tetrad(gam, x)
    dot = lambda a, b: np.einsum("i...,ij...,j...->...", a, gam, b)
    for a, b, v in [(rh, rh, 1), (th, th, 1), (ph, ph, 1), (rh, th, 0),
                    (rh, ph, 0), (th, ph, 0)]:
        assert np.allclose(dot(a, b), v, atol=1e-13)
    phit = np.array([-x[1], x[0], 0 * x[0]])
    # phihat along phi~ (same direction)
    cr = np.cross(ph.T, phit.T).T
    assert np.abs(cr).max() < 1e-13 and np.all(np.sum(ph * phit, 0) > 0)
    # rhat = a phi~ + b x with b > 0
    for k in range(npt):
        M = np.stack([phit[:, k], x[:, k]], 1)
        c, res, *_ = np.linalg.lstsq(M, rh[:, k], rcond=None)
        assert np.linalg.norm(M @ c - rh[:, k]) < 1e-13 and c[1] > 0
    # thetahat along sqrt(det) gamma^ik eps_klm phi~^l x^m, positively
    gi = np.moveaxis(np.linalg.inv(np.moveaxis(gam, (0, 1), (-2, -1))),
                     (-2, -1), (0, 1))
    tht = np.einsum("ik...,k...->i...", gi, np.cross(phit.T, x.T).T)
    assert np.all(dot(th, tht) > 0)


# ---- psi4_point against the 4-Riemann tensor --------------------------------------

@pytest.mark.parametrize("p", [(0.3, 0.5, -0.7, 0.2), (1.1, -0.4, 0.9, 0.6),
                               (-0.6, 1.3, 0.4, -1.2)])
def test_point_formula_pp_wave(ppw, p):
    gam = ppw.adm(p)[0]
    ref = S4.psi4_4d(ppw, p, _triad_at(gam, p[1:]))
    got = _psi4_3p1(ppw, p)
    assert abs(ref) > 1e-3
    assert abs(got - ref) <= 1e-12 * abs(ref)


@pytest.mark.parametrize("p", [(0.0, 3.0, 1.0, -2.0), (0.0, -2.5, 2.0, 1.5),
                               (0.0, 1.2, -2.2, 0.9)])
def test_point_formula_schwarzschild_off_centre(schw_off, p):
    gam = schw_off.adm(p)[0]
    ref = S4.psi4_4d(schw_off, p, _triad_at(gam, p[1:]))
    got = _psi4_3p1(schw_off, p)
    # the scale of the individual Riemann components is M / r^3
    scale = np.abs(schw_off.riemann_down(p)).max()
    assert abs(ref) > 1e-3 * scale
    assert abs(got - ref) <= 1e-12 * scale


def test_point_formula_schwarzschild_centred_is_zero():
    st = S4.schwarzschild_ks(M=1)
    for p in [(0.0, 3.0, 1.0, -2.0), (0.0, -1.5, 2.0, 0.7)]:
        scale = np.abs(st.riemann_down(p)).max()
        assert abs(_psi4_3p1(st, p)) <= 1e-13 * scale


# ---- the grid function ---------------------------------------------------------------

def _grid(n, lo, hi, ghost):
    return I.cell_centred(n, lo, hi, ghost)


def _poly_state(grid, seed):
    """phi = const, cubic gt_ij and At_ij, linear K (sympy expressions), so
    gamma_ij is cubic and K_ij of degree 4, both differentiated exactly by
    the stencils; and the state buffer holding them at every storage
    point."""
    rng = np.random.default_rng(seed)
    x, y, z = sympy.symbols("x y z")

    def cubic(base, amp, deg=3):
        p = sympy.Rational(base)
        for e in [(a, b, c) for a in range(4) for b in range(4)
                  for c in range(4) if a + b + c <= deg]:
            p += sympy.Rational(amp) * sympy.Rational(
                int(rng.integers(-64, 65)), 64) / (1 + sum(e))**2 * \
                x**e[0] * y**e[1] * z**e[2]
        return p

    phi = sympy.Rational("0.07")
    gt = [cubic("1.2" if i == j else "0.05", "0.04")
          for i, j in P.SYM]
    trK = cubic("0.2", "0.2", deg=1)  # gt_ij K stays of degree 4
    At = [cubic("0.1", "0.2") for _ in P.SYM]
    u = grid.empty()
    v = grid.view(u)
    X, Y, Z = grid.mesh()
    f = lambda e: np.broadcast_to(
        np.asarray(sympy.lambdify((x, y, z), e, "numpy")(X, Y, Z), float),
        X.shape)
    v[I.PHI] = float(phi)
    for c in range(6):
        v[I.GXX + c] = f(gt[c])
        v[I.AXX + c] = f(At[c])
    v[I.TRK] = f(trK)
    e4 = sympy.exp(4 * phi)
    gam = [e4 * gt[c] for c in range(6)]
    K = [e4 * (At[c] + gt[c] * trK / 3) for c in range(6)]
    return u, (x, y, z), gam, K


def _exact_inputs(xyz, gam6, K6, X, Y, Z):
    """gamma, its first and second derivatives, K and its first derivatives
    at the points (X, Y, Z), from the sympy expressions."""
    ev = lambda e: np.broadcast_to(
        np.asarray(sympy.lambdify(xyz, e, "numpy")(X, Y, Z), float), X.shape)
    sh = X.shape
    gam = np.zeros((3, 3) + sh)
    K = np.zeros((3, 3) + sh)
    dg = np.zeros((3, 3, 3) + sh)
    ddg = np.zeros((3, 3, 3, 3) + sh)
    dK = np.zeros((3, 3, 3) + sh)
    for c, (i, j) in enumerate(P.SYM):
        gam[i, j] = gam[j, i] = ev(gam6[c])
        K[i, j] = K[j, i] = ev(K6[c])
        for a in range(3):
            dg[a, i, j] = dg[a, j, i] = ev(sympy.diff(gam6[c], xyz[a]))
            dK[a, i, j] = dK[a, j, i] = ev(sympy.diff(K6[c], xyz[a]))
            for b in range(3):
                ddg[a, b, i, j] = ddg[a, b, j, i] = ev(
                    sympy.diff(gam6[c], xyz[a], xyz[b]))
    return gam, dg, ddg, K, dK


def _interior_mesh(grid):
    g = grid.ghost
    X, Y, Z = grid.mesh()
    s = (slice(g, g + grid.n[2]), slice(g, g + grid.n[1]),
         slice(g, g + grid.n[0]))
    return X[s], Y[s], Z[s]


@pytest.mark.parametrize("order,ghost", [(4, 3), (8, 5)])
def test_grid_polynomial_data_exact(order, ghost):
    grid = _grid((9, 7, 6), 0.3, 1.5, ghost)
    u, xyz, gam6, K6 = _poly_state(grid, 11 + order)
    centre = (0.1, -0.2, 0.05)
    got = P.psi4(grid, order, u, centre)
    X, Y, Z = _interior_mesh(grid)
    ex = _exact_inputs(xyz, gam6, K6, X, Y, Z)
    xr = np.array([X - centre[0], Y - centre[1], Z - centre[2]])
    ref = P.psi4_point(*ex, xr)
    scale = np.abs(ref).max()
    assert scale > 1e-2
    assert np.abs(got - ref).max() <= 2e-11 * scale


def test_grid_minkowski_is_exactly_zero():
    grid = _grid(8, -1.0, 1.0, 3)
    u = I.minkowski(grid) if hasattr(I, "minkowski") else None
    if u is None:
        u = grid.empty()
        v = grid.view(u)
        for c, (i, j) in enumerate(P.SYM):
            v[I.GXX + c] = 1.0 if i == j else 0.0
    out = P.psi4(grid, 4, u)
    assert np.all(out == 0)


def test_grid_flat_curvilinear_is_zero():
    """gamma_ij = d_i X^a d_j X^a for the quadratic map X = x + eps q(x):
    flat, with polynomial components of degree 2, K = 0."""
    grid = _grid((10, 9, 8), 0.4, 1.6, 3)
    x, y, z = sympy.symbols("x y z")
    eps = sympy.Rational(1, 10)
    Xm = [x + eps * (x * y - z * z / 2), y + eps * (x * z + y * y / 3),
          z + eps * (x * x - y * z)]
    J = sympy.Matrix(3, 3, lambda a, i: sympy.diff(Xm[a], (x, y, z)[i]))
    G = (J.T * J).applyfunc(sympy.expand)
    u = grid.empty()
    v = grid.view(u)
    Xg, Yg, Zg = grid.mesh()
    for c, (i, j) in enumerate(P.SYM):
        v[I.GXX + c] = np.broadcast_to(np.asarray(sympy.lambdify(
            (x, y, z), G[i, j], "numpy")(Xg, Yg, Zg), float), Xg.shape)
    out = P.psi4(grid, 4, u)
    # the curvature terms are O(eps^2) ~ 1e-2 each; they cancel to rounding
    assert np.abs(out).max() < 1e-13


def _pp_state(grid, st, t):
    """BSSN slots phi, gt, K, At of the pp-wave slice at time t (the paper's
    definitions: phi = ln(det gamma)/12, gt = e^{-4phi} gamma,
    K = gamma^ij K_ij, At = e^{-4phi}(K_ij - gamma_ij K/3))."""
    u = grid.empty()
    v = grid.view(u)
    X, Y, Z = grid.mesh()
    gam, K = st.adm_fields(t, X, Y, Z)
    gm = np.moveaxis(gam, (0, 1), (-2, -1))
    det = np.linalg.det(gm)
    gi = np.moveaxis(np.linalg.inv(gm), (-2, -1), (0, 1))
    phi = np.log(det) / 12.0
    trK = np.einsum("ij...,ij...->...", gi, K)
    v[I.PHI] = phi
    v[I.TRK] = trK
    for c, (i, j) in enumerate(P.SYM):
        v[I.GXX + c] = np.exp(-4 * phi) * gam[i, j]
        v[I.AXX + c] = np.exp(-4 * phi) * (K[i, j] - gam[i, j] * trK / 3)
    return u


def test_grid_pp_wave_fourth_order(ppw):
    t = 0.4
    errs = []
    for n in (12, 24):
        grid = _grid(n, 0.6, 1.1, 3)
        u = _pp_state(grid, ppw, t)
        got = P.psi4(grid, 4, u)
        X, Y, Z = _interior_mesh(grid)
        ex = ppw.adm_arrays(t, X, Y, Z)
        ref = P.psi4_point(*ex, np.array([X, Y, Z]))
        errs.append(np.abs(got - ref).max() / np.abs(ref).max())
    ratio = errs[0] / errs[1]
    assert errs[1] < 1e-7
    assert 13.0 < ratio < 18.0, (errs, ratio)
