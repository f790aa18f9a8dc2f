"""Pins of the oracle's constraint-norm reduction (no GPU).

The "L2 norm" of a constraint is read as the root mean square over the
interior points that are used, with |M| and |G| the flat Euclidean
magnitudes; the maxima are reported too.  Points at a distance <= r_exc
from any given centre are left out (N_used counts the rest), and a point
whose H, |M| or |G| is not finite is counted in N_nonfinite instead of
entering the sums.

The state is flat (gt = delta, phi = 0, A~ = 0, alpha = 1, beta = B = 0)
with K = k0 + c x and a constant evolved Gt^x = g0, so the constraints have
closed forms at every point: the Ricci terms vanish (every metric
derivative is exactly zero), H = (2/3) K^2, M = (-(2/3) c, 0, 0) (the
centred first difference is exact on a linear function), G = (g0, 0, 0).
The grid has spacing 1/2 on dyadic coordinates, so the face neighbours of a
centre on a grid point lie exactly at r_exc = 1/2 and the diagonal ones at
sqrt(1/2): the excised sets are countable by hand, and a strict '<' in
place of '<=' changes N_used (and the RMS) by the six face neighbours.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1111_3344_amd import inputs as I

K0, C, G0 = 1.0, 0.25, 0.375
N = 7
ORIGIN = -1.5  # interior coordinates -1.5, -1.0, ..., 1.5 on every axis


def _grid():
    return I.GridSpec((N, N, N), 3, (0.5, 0.5, 0.5), (ORIGIN,) * 3,
                      I.BC_STATIC)


def _state(g):
    u = I.minkowski(g)
    X, _, _ = g.mesh()
    g.view(u)[I.TRK] = K0 + C * X
    g.view(u)[I.GAMX] = G0
    return u


def _coords():
    ax = ORIGIN + 0.5 * np.arange(N)
    Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")  # [z][y][x]
    return X, Y, Z


def _closed_form_norms(used):
    """The 8 norms from the closed forms over the boolean mask `used`
    ([z][y][x] interior points)."""
    X, _, _ = _coords()
    H = (2.0 / 3.0) * (K0 + C * X) ** 2
    n = int(used.sum())
    return np.array([np.sqrt((H[used] ** 2).sum() / n), np.abs(H[used]).max(),
                     (2.0 / 3.0) * C, (2.0 / 3.0) * C, G0, G0, n, 0.0])


def _check(norms, ref, nonfinite=0):
    assert norms[6] == ref[6], ("N_used", norms[6], ref[6])
    assert norms[7] == nonfinite, ("N_nonfinite", norms[7])
    np.testing.assert_allclose(norms[:6], ref[:6], rtol=1e-13, atol=0)


def test_no_mask_uses_every_interior_point():
    g = _grid()
    _, _, _, n = O.constraints(g, O.params(), _state(g))
    ref = _closed_form_norms(np.ones((N, N, N), bool))
    assert ref[6] == N ** 3
    _check(n, ref)


def test_fields_have_their_closed_forms():
    g = _grid()
    H, M, Gc, _ = O.constraints(g, O.params(), _state(g))
    X, _, _ = _coords()
    np.testing.assert_allclose(g.interior(H, 1)[0], (2 / 3) * (K0 + C * X) ** 2,
                               rtol=1e-14, atol=0)
    m = g.interior(M, 3)
    np.testing.assert_allclose(m[0], -(2 / 3) * C, rtol=1e-13, atol=0)
    assert np.abs(m[1:]).max() == 0.0
    gc = g.interior(Gc, 3)
    assert (gc[0] == G0).all() and np.abs(gc[1:]).max() == 0.0


def test_mask_by_hand_geometry_one_centre():
    """Centre on the grid point (0, 0, 0) (index 3, 3, 3), r_exc = 1/2: the
    centre and its six face neighbours (at exactly 1/2) are left out,
    the twelve edge neighbours (at sqrt(1/2)) are kept."""
    g = _grid()
    _, _, _, n = O.constraints(g, O.params(), _state(g), [(0.0, 0.0, 0.0)],
                               0.5)
    used = np.ones((N, N, N), bool)
    for d in [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
              (0, 0, 1), (0, 0, -1)]:
        used[3 + d[2], 3 + d[1], 3 + d[0]] = False
    ref = _closed_form_norms(used)
    assert ref[6] == N ** 3 - 7
    _check(n, ref)


def test_mask_by_hand_geometry_two_centres():
    """Centres at (0, 0, 0) and (1/2, 0, 0), neighbours of each other: the
    union of the two excised sets has 7 + 7 - 2 = 12 points."""
    g = _grid()
    cent = [(0.0, 0.0, 0.0), (0.5, 0.0, 0.0)]
    _, _, _, n = O.constraints(g, O.params(), _state(g), cent, 0.5)
    used = np.ones((N, N, N), bool)
    for cx in (3, 4):
        for d in [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
                  (0, 0, 1), (0, 0, -1)]:
            used[3 + d[2], 3 + d[1], cx + d[0]] = False
    ref = _closed_form_norms(used)
    assert ref[6] == N ** 3 - 12
    _check(n, ref)


def test_nonfinite_points_counted_not_summed():
    """K = NaN at interior point (5, 1, 1): H is NaN there, and M at every
    point whose first-difference stencil (offsets +-1, +-2 along an axis)
    reaches it: (4,1,1), (6,1,1), (3,1,1) [(7,1,1) is outside], (5,0,1),
    (5,2,1), (5,3,1) [(5,-1,1) outside], and likewise in z: 10 points,
    none near the centres.  They are counted, and the sums and maxima are
    those of the other points."""
    g = _grid()
    u = _state(g)
    g.interior(u)[I.TRK, 1, 1, 5] = np.nan  # [slot][z][y][x]
    cent = [(0.0, 0.0, 0.0), (0.5, 0.0, 0.0)]
    _, _, _, n = O.constraints(g, O.params(), u, cent, 0.5)
    used = np.ones((N, N, N), bool)
    for cx in (3, 4):
        for d in [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
                  (0, 0, 1), (0, 0, -1)]:
            used[3 + d[2], 3 + d[1], cx + d[0]] = False
    bad = [(5, 1, 1), (4, 1, 1), (6, 1, 1), (3, 1, 1), (5, 0, 1), (5, 2, 1),
           (5, 3, 1), (5, 1, 0), (5, 1, 2), (5, 1, 3)]
    for x, y, z in bad:
        used[z, y, x] = False
    ref = _closed_form_norms(used)
    assert ref[6] == N ** 3 - 12 - 10
    _check(n, ref, nonfinite=10)
    assert np.isfinite(n).all()


@pytest.mark.parametrize("r_exc", [0.0, 0.49])
def test_mask_radius_below_the_spacing_excises_only_the_centre(r_exc):
    """r_exc below the spacing leaves out the centre point alone (distance
    0 <= r_exc), and with r_exc = 0 still the centre."""
    g = _grid()
    _, _, _, n = O.constraints(g, O.params(), _state(g), [(0.0, 0.0, 0.0)],
                               r_exc)
    used = np.ones((N, N, N), bool)
    used[3, 3, 3] = False
    _check(n, _closed_form_norms(used))
