"""Psi_4 on the GPU (bssn_psi4) against the oracle (oracle/psi4.py),
through the C ABI (needs an MI355X).

Tolerance.  Both sides evaluate the same stencils and algebra in FP64 in a
different order (the kernel contracts the six Riemann pair components with
the tetrad bivector, the oracle the full 81-component tensor).  The
dominant rounding is that of the second differences: each is a sum of
about 2 order/2 + 1 values of |g| <= G with weights of total size
W2 = 2 sum|b_k| + 2 sum b_k (< 6 at order 4, < 7 at order 8), divided by
h^2, so it carries an absolute error of a few W2 eps G / h^2; Psi_4 is a
combination of the second derivatives with coefficients of order one (the
tetrad's vectors are unit vectors of g, their components at most ~2), so
    |Psi4_gpu - Psi4_oracle| <= 8 W2 eps G / h^2 + 1e-13 max|Psi4|,
the second term for the first-derivative and product parts.  The tests
print the largest error over this bound (about 0.01 when first run) and
the error relative to max |Psi4|.
"""
import math

import numpy as np
import pytest

from oracle import multipole as MP
from oracle import psi4 as P
from paper_1111_3344_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = np.finfo(float).eps
W2 = {4: 2 * (4 / 3 + 1 / 12) * 2, 8: 2 * (8 / 5 + 1 / 5 + 8 / 315 + 1 / 560) * 2}
SENTINEL = 7.25


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1111_3344_amd import bssn
    bssn.lib()
    return bssn


def _gmax(grid, u):
    v = grid.view(u)
    e4 = np.exp(4 * v[I.PHI])
    return max(np.abs(e4 * v[I.GXX + c]).max() for c in range(6))


def _bound(grid, u, order, ref):
    return (8 * W2[order] * EPS * _gmax(grid, u) / min(grid.h) ** 2
            + 1e-13 * np.abs(ref).max())


def _gpu(B, grid, order, u, centre):
    out = torch.full((grid.off0 + 2 * grid.sf,), SENTINEL,
                     dtype=torch.float64, device="cuda")
    B.bssn_psi4(grid, order, B.to_device(u), out, centre)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    v = grid.view(o, nslot=2)
    return v, grid.interior(o, nslot=2)


CASES = {
    # name: (n, ghost, order, h, seed)
    "o4-several-tiles-ragged": ((37, 11, 9), 3, 4, 0.25, 71),
    "o8-several-tiles-ragged": ((35, 9, 10), 5, 8, 0.25, 72),
    "o4-one-point": ((1, 1, 1), 3, 4, 0.3, 73),
    "o8-thin": ((17, 1, 5), 5, 8, 0.2, 74),
    "o4-wide-ghost": ((20, 6, 7), 5, 4, 0.2, 75),
}
CENTRE = (0.013, -0.021, 0.007)


@pytest.mark.parametrize("case", list(CASES))
def test_psi4_matches_oracle(B, case):
    n, ghost, order, h, seed = CASES[case]
    origin = tuple(-0.5 * n[a] * h + 0.37 * h for a in range(3))
    grid = I.GridSpec(n, ghost, (h,) * 3, origin, I.BC_STATIC)
    u = I.smooth_random(grid, seed=seed)
    print(f"[psi4] {case}", flush=True)
    want = P.psi4(grid, order, u, CENTRE)
    full, got = _gpu(B, grid, order, u, CENTRE)
    err = np.maximum(np.abs(got[0] - want.real), np.abs(got[1] - want.imag))
    bound = _bound(grid, u, order, want)
    print(f"[psi4] {case}: max |Psi4| = {np.abs(want).max():.3e}, "
          f"max error / bound = {err.max() / bound:.3f}, "
          f"/ max |Psi4| = {err.max() / np.abs(want).max():.2e}", flush=True)
    assert np.isfinite(got).all()
    assert err.max() <= bound
    # nothing outside the interior is written
    g = grid.ghost
    mask = np.ones(full.shape[1:], bool)
    mask[g:g + n[2], g:g + n[1], g:g + n[0]] = False
    assert np.all(full[:, mask] == SENTINEL)


def test_minkowski_is_zero(B):
    grid = I.cell_centred((19, 6, 5), -1.0, 1.0, 3)
    u = I.minkowski(grid)
    _, got = _gpu(B, grid, 4, u, CENTRE)
    assert np.all(got == 0)


def test_multipole_of_psi4(B):
    """Multipole (spin -2) of the kernel's Psi_4 against the oracle's
    multipole of the oracle's Psi_4: the two analysis modules chained."""
    n, h = (24, 22, 21), 0.2
    origin = tuple(-0.5 * n[a] * h + 0.5 * h for a in range(3))
    grid = I.GridSpec(n, 3, (h,) * 3, origin, I.BC_STATIC)
    u = I.smooth_random(grid, seed=77)
    want_psi = P.psi4(grid, 4, u, CENTRE)
    re = grid.empty()[:grid.off0 + grid.sf].copy()
    im = re.copy()
    grid.interior(re, nslot=1)[0] = want_psi.real
    grid.interior(im, nslot=1)[0] = want_psi.imag
    # the sphere stays inside the interior: ghosts are never read
    want = MP.multipole(grid, grid.view(re, nslot=1)[0],
                        grid.view(im, nslot=1)[0], CENTRE, 1.4, -2, 4, 12, 24)
    out = torch.zeros(grid.off0 + 2 * grid.sf, dtype=torch.float64,
                      device="cuda")
    B.bssn_psi4(grid, 4, B.to_device(u), out, CENTRE)
    got = B.bssn_multipole(grid, out, out, CENTRE, 1.4, -2, 4, 12, 24,
                           re_slot=0, im_slot=1)
    scale = np.abs(want).max()
    err = np.abs(got - want).max() / scale
    print(f"[psi4] multipole: max |C| = {scale:.3e}, "
          f"max error / max |C| = {err:.2e}", flush=True)
    assert scale > 1e-3
    assert err <= 1e-10


def _sub_oracle(grid, u, order, lo, size, centre):
    """Oracle Psi_4 on the interior box [lo, lo + size) of a large grid,
    from a sub-grid holding the box and order/2 points around it."""
    M = order // 2
    sub = I.GridSpec(tuple(size), M, grid.h,
                     tuple(grid.origin[a] + lo[a] * grid.h[a]
                           for a in range(3)), I.BC_STATIC)
    us = sub.empty()
    g = grid.ghost
    src = grid.view(u)[:, g + lo[2] - M:g + lo[2] + size[2] + M,
                       g + lo[1] - M:g + lo[1] + size[1] + M,
                       g + lo[0] - M:g + lo[0] + size[0] + M]
    sub.view(us)[...] = src
    return P.psi4(sub, order, us, centre), sub, us


@pytest.mark.parametrize("order,n,ghost", [(4, 128, 3), (8, 96, 5)])
def test_full_size_sampled(B, order, n, ghost):
    """The 128^3 grid on [-8, 8]^3 (and 96^3 at order 8) holding two
    Brill-Lindquist punctures after two RK4 steps on the GPU (non-zero K and
    A~), every point's Psi_4 computed by the kernel; the oracle on boxes at
    the corners, faces, the punctures and the centre."""
    grid = I.cell_centred(n, -8.0, 8.0, ghost)
    u0 = I.brill_lindquist(grid, (0.5, 0.5), ((3.0, 0, 0), (-3.0, 0, 0)))
    prm = B.Params(fd_order=order)
    du = B.to_device(u0)
    a, b, acc = (B.empty_state(grid) for _ in range(3))
    a.copy_(du)
    b.copy_(du)
    acc.copy_(du)
    for _ in range(2):
        B.rk4_step(grid, prm, 0.03125, du, a, b, acc)
    torch.cuda.synchronize()
    u = du.cpu().numpy()
    print(f"[psi4] full size order {order}, n = {n}", flush=True)
    _, got = _gpu(B, grid, order, u, CENTRE)
    assert np.isfinite(got).all()
    size = (6, 5, 4)
    lows = [(0, 0, 0), (n - 6, n - 5, n - 4), (0, n // 2, n - 4),
            (n // 2 - 3, n // 2 - 2, n // 2 - 2), (n - 6, 0, n // 2),
            (int(n * 11 / 16) - 3, n // 2 - 2, n // 2 - 2),
            (int(n * 5 / 16) - 3, n // 2 - 3, n // 2 - 1)]
    worst = rel = 0.0
    for lo in lows:
        want, sub, us = _sub_oracle(grid, u, order, lo, size, CENTRE)
        sl = (slice(lo[2], lo[2] + size[2]), slice(lo[1], lo[1] + size[1]),
              slice(lo[0], lo[0] + size[0]))
        err = np.maximum(np.abs(got[0][sl] - want.real),
                         np.abs(got[1][sl] - want.imag)).max()
        bound = _bound(sub, us, order, want)
        worst = max(worst, err / bound)
        rel = max(rel, err / np.abs(want).max())
        assert err <= bound, (lo, err, bound)
    print(f"[psi4] full size order {order}: max error / bound = {worst:.3f},"
          f" max error / max |Psi4| of its box = {rel:.2e}", flush=True)
