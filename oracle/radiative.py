"""Radiative (Sommerfeld-type) outer boundary of the BSSN right-hand side,
plain numpy in FP64.  Test infrastructure only.

It follows the boundary-conditions subsection of the paper's spacetime
curvature evolution section. Near the outer boundary every evolved
component X is taken to behave as an outgoing spherical wave
X = X0 + u(r - v0 t) / r. That gives the wave part of its source,
    S = -v^i d_i X - v0 (X - X0) / r,   v^i = v0 x^i / r,
with second-order differences: centred where both neighbours exist,
one-sided at the edge of the storage grid.

The part of the source that is not such a wave is assumed to fall off as
r^-p (p = 2). It is carried outward from the neighbouring point one layer
further in. The boundary points are the ghost layers of a static grid,
evaluated layer by layer starting at the innermost.

Readings (the printed correction formula is garbled):
  * layer k (1 .. ghost): the storage points whose largest per-axis
    distance outside the interior box is k; layer 0 is the interior;
  * n: the outward normal of the point's face, edge or corner, one
    component in {-1, 0, +1} per axis; the inward neighbour q = p - n lies
    in layer k - 1;
  * rhs(p) = S(p) + (r_q / r_p)^p (rhs(q) - S(q)): the non-wave part at q,
    decayed by the power law from r_q to r_p;
  * x^i are coordinates relative to the coordinate origin, r = |x|.
"""
import numpy as np

NSLOT = 25


def storage_coords(grid):
    """Coordinates (z, y, x order of the storage arrays) of every storage
    point: x_a(j) = origin_a + (j - ghost) h_a."""
    g = grid.ghost
    ax = [grid.origin[a] + (np.arange(grid.n[a] + 2 * g) - g) * grid.h[a]
          for a in range(3)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return X, Y, Z


def deriv(f, axis, h):
    """Second-order first derivative of f (..., Z, Y, X) along storage axis
    `axis` (0 = x, 1 = y, 2 = z): centred inside, one-sided (three points)
    at the two ends."""
    ax = f.ndim - 1 - axis
    f = np.moveaxis(f, ax, -1)
    d = np.empty_like(f)
    d[..., 1:-1] = (f[..., 2:] - f[..., :-2]) / (2 * h)
    d[..., 0] = (-3 * f[..., 0] + 4 * f[..., 1] - f[..., 2]) / (2 * h)
    d[..., -1] = (3 * f[..., -1] - 4 * f[..., -2] + f[..., -3]) / (2 * h)
    return np.moveaxis(d, -1, ax)


def wave_part(grid, u, x0, v0):
    """S at every storage point, shape (25, Z, Y, X)."""
    v = grid.view(u)
    X, Y, Z = storage_coords(grid)
    r = np.sqrt(X * X + Y * Y + Z * Z)
    x0 = np.asarray(x0, float).reshape(NSLOT, 1, 1, 1)
    v0 = np.asarray(v0, float).reshape(NSLOT, 1, 1, 1)
    xd = (X * deriv(v, 0, grid.h[0]) + Y * deriv(v, 1, grid.h[1]) +
          Z * deriv(v, 2, grid.h[2]))
    return -v0 * xd / r - v0 * (v - x0) / r


def layers(grid):
    """Per storage point: its layer (0 inside) and its outward normal."""
    g = grid.ghost
    side, dist = [], []
    for a in range(3):
        j = np.arange(grid.n[a] + 2 * g)
        s = np.where(j < g, -1, np.where(j >= grid.n[a] + g, 1, 0))
        d = np.where(j < g, g - j, np.where(j >= grid.n[a] + g,
                                            j - (grid.n[a] + g - 1), 0))
        side.append(s)
        dist.append(d)
    layer = np.maximum(np.maximum(dist[2][:, None, None],
                                  dist[1][None, :, None]),
                       dist[0][None, None, :])
    return layer, side


def radiative_rhs(grid, u, rhs, x0, v0, p=2):
    """rhs with its ghost layers set by the radiative condition; the
    interior of rhs (the evolved points' right-hand side) is read, not
    changed."""
    out = np.array(rhs, dtype=np.float64, copy=True)
    ov = grid.view(out)
    S = wave_part(grid, u, x0, v0)
    X, Y, Z = storage_coords(grid)
    r = np.sqrt(X * X + Y * Y + Z * Z)
    layer, side = layers(grid)
    for k in range(1, grid.ghost + 1):
        zi, yi, xi = np.nonzero(layer == k)
        qz, qy, qx = zi - side[2][zi], yi - side[1][yi], xi - side[0][xi]
        f = (r[qz, qy, qx] / r[zi, yi, xi]) ** p
        ov[:, zi, yi, xi] = S[:, zi, yi, xi] + f * (ov[:, qz, qy, qx] -
                                                   S[:, qz, qy, qx])
    return out
