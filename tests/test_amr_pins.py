"""Pins of the mesh-refinement oracle (oracle/amr.py) on the CPU:
  * the interpolation weights are the textbook ones: (-7, 105, 35, -5)/128
    at a quarter spacing (cell-centred 2:1 prolongation) and
    (-1, 9, 9, -1)/16 at the midpoint (restriction);
  * prolongation is exact for a field that is a cubic in each coordinate,
    on faces, edges and corners of every fine patch, also where the coarse
    block comes from the ghosts of a coarse patch or from the second coarse
    patch across a seam, and on a third level;
  * interpolation in time is exact for a quadratic in t (three levels) and
    a line (two levels);
  * a ghost point inside a sibling's interior takes the sibling's value
    (a copy, checked by hand geometry), every other ghost the coarse one;
    on level 0 the shared face is exchanged and the physical boundary
    ghosts are left alone;
  * restriction is exact for a tricubic field on the covered coarse points
    and leaves every other point alone;
  * prolongation of a smooth field converges at fourth order;
  * an uncovered ghost point is an error.
"""
import numpy as np
import pytest

from oracle import amr as M
from paper_1111_3344_amd import inputs as I
from tests import amr_hier as H


def _poly(X, Y, Z, s):
    return ((1.0 + 0.1 * s) * (0.5 - 0.3 * X + 0.2 * X ** 3) *
            (1.0 + 0.4 * Y - 0.1 * Y ** 2 + 0.05 * Y ** 3) +
            0.3 * X * Y * Z ** 3 - 0.2 * Z ** 2 + 0.01 * s * Z)


def _fill(g, fn):
    u = g.empty()
    v = g.view(u)
    X, Y, Z = g.mesh()
    for s in range(25):
        v[s] = fn(X, Y, Z, s)
    return u


def _ghost_mask(g):
    m = np.ones(tuple(g.ext[::-1]), bool)
    c = g.ghost
    m[c:-c, c:-c, c:-c] = False
    return m


def test_textbook_weights():
    assert np.allclose(M.lagrange(1.25, [0, 1, 2, 3]),
                       np.array([-7, 105, 35, -5]) / 128, rtol=0, atol=1e-16)
    assert np.allclose(M.lagrange(1.75, [0, 1, 2, 3]),
                       np.array([-5, 35, 105, -7]) / 128, rtol=0, atol=1e-16)
    assert np.allclose(M.lagrange(1.5, [0, 1, 2, 3]),
                       np.array([-1, 9, 9, -1]) / 16, rtol=0, atol=1e-16)


@pytest.mark.parametrize("hier", [H.two_level, H.three_level])
def test_prolongation_exact_for_tricubic(hier):
    hr = hier()
    states = [_fill(g, _poly) for _, g in hr]
    top = max(lv for lv, _ in hr)
    for level in range(1, top + 1):
        for p, (lv, g) in enumerate(hr):
            if lv == level:
                g.view(states[p])[:, _ghost_mask(g)] = 0.0
        M.fill_ghosts(hr, level, states, [states], [0.0], 0.0)
    for p, (lv, g) in enumerate(hr):
        want = g.view(_fill(g, _poly))
        got = g.view(states[p])
        assert np.allclose(got, want, rtol=1e-13, atol=1e-13), p


def test_time_interpolation_exact():
    hr = H.two_level()
    q2 = lambda t: 1.0 - 0.3 * t + 0.2 * t * t
    q1 = lambda t: 0.7 + 0.4 * t
    for q, ts, t in ((q2, [0.0, 0.5, 1.0], 0.75), (q2, [-1.0, 0.0, 1.0], 0.25),
                     (q1, [0.0, 1.0], 0.5)):
        levels = [[_fill(g, lambda X, Y, Z, s: _poly(X, Y, Z, s) * q(tl))
                   for _, g in hr] for tl in ts]
        states = [u.copy() for u in levels[0]]
        M.fill_ghosts(hr, 1, states, levels, ts, t)
        for p, (lv, g) in enumerate(hr):
            if lv != 1:
                continue
            m = _ghost_mask(g)
            got = g.view(states[p])[:, m]
            want = g.view(_fill(g, _poly))[:, m] * q(t)
            # ghosts copied from a sibling hold the sibling's first level
            cp = _copied(hr, p)
            want[:, cp[m]] = g.view(_fill(g, _poly))[:, m][:, cp[m]] * q(ts[0])
            assert np.allclose(got, want, rtol=1e-13, atol=1e-13)


def _copied(hr, p):
    """Ghost points of patch p that lie in another same-level interior, by
    coordinates (the test's own geometry)."""
    lv, g = hr[p]
    X, Y, Z = g.mesh()
    out = np.zeros(X.shape, bool)
    for q, (lq, gq) in enumerate(hr):
        if q == p or lq != lv:
            continue
        inside = np.ones(X.shape, bool)
        for a, C in enumerate((X, Y, Z)):
            lo = gq.origin[a] - 0.5 * gq.h[a]
            hi = gq.origin[a] + (gq.n[a] - 0.5) * gq.h[a]
            inside &= (C > lo) & (C < hi)
        out |= inside
    return out & _ghost_mask(g)


def test_sibling_copy_before_prolongation():
    hr = H.two_level()
    states = [_fill(g, _poly) for _, g in hr]
    # fine interiors get a per-patch offset, ghosts are cleared
    for p, (lv, g) in enumerate(hr):
        if lv == 1:
            v = g.view(states[p])
            v[:, g.ghost:-g.ghost, g.ghost:-g.ghost, g.ghost:-g.ghost] += \
                100.0 * p
            v[:, _ghost_mask(g)] = 0.0
    M.fill_ghosts(hr, 1, states, [states], [0.0], 0.0)
    # f0 (patch 2) and f1 (patch 3) touch at f0's +x face: f0's +x ghosts
    # whose y and z lie in f1's interior hold f1's values
    g0 = hr[2][1]
    c = g0.ghost
    v = g0.view(states[2])
    P = g0.view(_fill(g0, _poly))
    ny, nz = g0.n[1], g0.n[2]
    xs = slice(c + g0.n[0], 2 * c + g0.n[0])
    inner = v[:, c:c + nz, c:c + ny, xs]
    assert np.allclose(inner, P[:, c:c + nz, c:c + ny, xs] + 300.0,
                       rtol=1e-14, atol=1e-12)
    # an edge ghost there (y below f1's interior) is prolonged
    assert np.allclose(v[:, c, c - 1, xs], P[:, c, c - 1, xs], rtol=1e-13,
                       atol=1e-13)
    # the copied set found by coordinates equals the points that carry an
    # offset
    cp = _copied(hr, 2)
    assert cp.sum() == g0.ghost * ny * nz
    got_off = np.abs(v[0] - P[0]) > 50
    assert np.array_equal(got_off & _ghost_mask(g0), cp)


def test_level0_sync_copies_and_keeps_the_boundary():
    hr = H.two_level()
    rng = np.random.default_rng(12)
    states = [rng.normal(size=g.total) for _, g in hr]
    before = [u.copy() for u in states]
    M.fill_ghosts(hr, 0, states, None, None, 0.0)
    # c0 (patch 0) and c1 (patch 1) touch at c0's +x face
    c0, c1 = hr[0][1], hr[1][1]
    g = c0.ghost
    v0, v1 = c0.view(states[0]), c1.view(states[1])
    face = v0[:, g:-g, g:-g, g + c0.n[0]:]
    assert np.array_equal(face, v1[:, g:-g, g:-g, g:2 * g])
    face1 = v1[:, g:-g, g:-g, :g]
    assert np.array_equal(face1, v0[:, g:-g, g:-g, c0.n[0]:c0.n[0] + g])
    # every other point of the level-0 patches is unchanged, and the fine
    # patches are not touched
    m0 = np.zeros(v0.shape[1:], bool)
    m0[g:-g, g:-g, g + c0.n[0]:] = True
    assert np.array_equal(v0[:, ~m0], c0.view(before[0])[:, ~m0])
    m1 = np.zeros(v1.shape[1:], bool)
    m1[g:-g, g:-g, :g] = True
    assert np.array_equal(v1[:, ~m1], c1.view(before[1])[:, ~m1])
    for p in range(2, len(hr)):
        assert np.array_equal(states[p], before[p])


def test_restriction_exact_and_local():
    hr = H.two_level()
    rng = np.random.default_rng(5)
    coarse = [None] * len(hr)
    fine = [None] * len(hr)
    for p, (lv, g) in enumerate(hr):
        if lv == 0:
            coarse[p] = rng.normal(size=g.total)
        else:
            fine[p] = _fill(g, _poly)
    before = [c.copy() if c is not None else None for c in coarse]
    M.restrict(hr, 1, fine, coarse)
    for p, (lv, g) in enumerate(hr):
        if lv != 0:
            continue
        X, Y, Z = g.mesh()
        cov = np.zeros(X.shape, bool)
        for q, (lq, fg) in enumerate(hr):
            if lq != 1:
                continue
            inside = np.ones(X.shape, bool)
            for a, C in enumerate((X, Y, Z)):
                lo = fg.origin[a] - 0.5 * fg.h[a]
                hi = fg.origin[a] + (fg.n[a] - 0.5) * fg.h[a]
                inside &= (C > lo) & (C < hi)
            cov |= inside
        cov &= ~_ghost_mask(g)
        assert cov.sum() > 0
        got, old = g.view(coarse[p]), g.view(before[p])
        want = g.view(_fill(g, _poly))
        assert np.allclose(got[:, cov], want[:, cov], rtol=1e-13, atol=1e-13)
        assert np.array_equal(got[:, ~cov], old[:, ~cov])


def test_prolongation_fourth_order():
    def smooth(X, Y, Z, s):
        return np.sin(0.9 * X + 0.3 * s) * np.cos(0.7 * Y - 0.4 * Z) + Z * X

    errs = []
    for h in (0.2, 0.1):
        c = I.GridSpec((int(2.4 / h),) * 3, 3, (h, h, h), (-1.2, -1.1, -1.3),
                       I.BC_STATIC)
        m = int(round(0.6 / h))
        f = H.child(c, (m, m, m), (int(1.2 / h),) * 3)
        hr = [(0, c), (1, f)]
        states = [_fill(c, smooth), f.empty()]
        M.fill_ghosts(hr, 1, states, [states], [0.0], 0.0)
        gm = _ghost_mask(f)
        errs.append(np.abs(f.view(states[1])[:, gm] -
                           f.view(_fill(f, smooth))[:, gm]).max())
    assert 12 < errs[0] / errs[1] < 20, errs


def test_uncovered_ghost_is_an_error():
    c = I.GridSpec((8, 8, 8), 3, (0.2,) * 3, (0.0, 0.0, 0.0), I.BC_STATIC)
    f = H.child(c, (-3, 0, 0), (8, 8, 8))      # sticks out of c at -x
    hr = [(0, c), (1, f)]
    with pytest.raises(ValueError):
        M.fill_ghosts(hr, 1, [c.empty(), f.empty()], [[c.empty(),
                      f.empty()]], [0.0], 0.0)
