"""Initial conversion from the ADM variables to the BSSN state, plain numpy
in FP64.  Test infrastructure only.

It follows the initial-conditions subsection of the paper's spacetime
curvature evolution section. The BSSN quantities come from their
definitions (the variables listed in the same section):
    phi = ln(det g) / 12,   gt_ij = e^{-4 phi} g_ij,   K = g^ij K_ij,
    At_ij = e^{-4 phi} (K_ij - g_ij K / 3),   B^i = 0,
with alpha and beta^i copied. The conformal connection
    Gt^i = gt^ij gt^kl Gt_jkl,   Gt_jkl = (d_l gt_jk + d_k gt_jl - d_j gt_kl)/2,
takes derivatives of the metric. They are centred differences of the
grid's order at interior points. On the ghost layers, where a centred
stencil would not fit, Gt^i is extrapolated with a cubic:
    X(p) = 4 X(p - n) - 6 X(p - 2n) + 4 X(p - 3n) - X(p - 4n).
Here n is the outward normal of p's face (perpendicular), or the sum of
the normals of the faces that meet at p's edge or corner, e.g. (1, 1, 0)
or (1, 1, 1). Layers are filled innermost first.

Readings:
  * the lapse time-derivative slot A is 0;
  * the derivatives of gt_ij are those of the converted field (a grid
    function), in the centre-relative pairwise form of the main kernels;
  * layer k is the set of storage points whose largest per-axis distance
    outside the interior box is k.

ADM input layout: 16 slots in the state layout (slot stride sf):
g_xx g_xy g_xz g_yy g_yz g_zz, K_xx K_xy K_xz K_yy K_yz K_zz, alpha,
beta^x beta^y beta^z.
"""
import numpy as np

from . import radiative as _rad

NSLOT = 25
PHI, GXX, TRK, AXX, GAMX, ALP, BETX, BX, ADOT = 0, 1, 7, 8, 14, 17, 18, 21, 24
# symmetric pair (i, j) -> 0..5 in the order xx xy xz yy yz zz
SYM = {(0, 0): 0, (0, 1): 1, (0, 2): 2, (1, 1): 3, (1, 2): 4, (2, 2): 5}
for (i, j), m in list(SYM.items()):
    SYM[(j, i)] = m

# centred first-derivative weights a(k) of the pairwise form
# d f = sum_k a(k) (f(k) - f(-k)) / h
FD_A = {4: (2.0 / 3.0, -1.0 / 12.0),
        8: (4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0)}


def _mat(s6):
    """(6, ...) symmetric components -> (3, 3, ...) matrix."""
    return np.array([[s6[SYM[(i, j)]] for j in range(3)] for i in range(3)])


def _det(m):
    return (m[0, 0] * (m[1, 1] * m[2, 2] - m[1, 2] * m[2, 1])
            - m[0, 1] * (m[1, 0] * m[2, 2] - m[1, 2] * m[2, 0])
            + m[0, 2] * (m[1, 0] * m[2, 1] - m[1, 1] * m[2, 0]))


def _inv(m):
    d = _det(m)
    inv = np.empty_like(m)
    for i in range(3):
        for j in range(3):
            a = [r for r in range(3) if r != j]
            b = [c for c in range(3) if c != i]
            minor = m[a[0], b[0]] * m[a[1], b[1]] - m[a[0], b[1]] * m[a[1], b[0]]
            inv[i, j] = (-1) ** (i + j) * minor / d
    return inv


def _deriv_interior(f, axis, h, order, g):
    """Centred derivative of f (..., Z, Y, X) along storage axis `axis`
    (0 = x) at the interior points, shape (..., nz, ny, nx)."""
    a = FD_A[order]
    ax = f.ndim - 1 - axis
    n = f.shape[ax] - 2 * g
    out = 0.0
    for k, w in enumerate(a, start=1):
        hi = np.take(f, np.arange(g + k, g + k + n), axis=ax)
        lo = np.take(f, np.arange(g - k, g - k + n), axis=ax)
        out = out + w * (hi - lo)
    out = out / h
    # restrict the other two axes to the interior
    sl = [slice(None)] * f.ndim
    for other in range(3):
        if other != axis:
            o = f.ndim - 1 - other
            sl[o] = slice(g, f.shape[o] - g)
    return out[tuple(sl)]


def extrapolate_layers(grid, field):
    """Fill the ghost layers of field (..., Z, Y, X) by cubic extrapolation
    along each point's normal, innermost layer first (in place)."""
    layer, side = _rad.layers(grid)
    for k in range(1, grid.ghost + 1):
        zi, yi, xi = np.nonzero(layer == k)
        nz, ny, nx = side[2][zi], side[1][yi], side[0][xi]
        pts = [field[..., zi - m * nz, yi - m * ny, xi - m * nx]
               for m in range(1, 5)]
        field[..., zi, yi, xi] = 4 * pts[0] - 6 * pts[1] + 4 * pts[2] - pts[3]
    return field


def from_adm(grid, adm, order=4):
    """BSSN state (flat, the shared layout) from the ADM variables (flat,
    16 slots in the same layout)."""
    a = grid.view(adm, 16)
    g6, k6 = a[0:6], a[6:12]
    gm = _mat(g6)
    det = _det(gm)
    phi = np.log(det) / 12.0
    e4 = np.exp(-4.0 * phi)
    gu = _inv(gm)
    trK = sum(gu[i, j] * k6[SYM[(i, j)]] for i in range(3) for j in range(3))
    out = grid.empty()
    v = grid.view(out)
    v[PHI] = phi
    for m in range(6):
        v[GXX + m] = e4 * g6[m]
        v[AXX + m] = e4 * (k6[m] - g6[m] * trK / 3.0)
    v[TRK] = trK
    v[ALP] = a[12]
    for i in range(3):
        v[BETX + i] = a[13 + i]
        v[BX + i] = 0.0
    v[ADOT] = 0.0
    # conformal connection at interior points from the converted metric
    gc = grid.ghost
    gt = v[GXX:GXX + 6]
    dg = [_deriv_interior(gt, ax, grid.h[ax], order, gc) for ax in range(3)]
    gti = gt[:, gc:-gc, gc:-gc, gc:-gc]
    gtu = _inv(_mat(gti))
    # Gl[j][k][l] = (d_l gt_jk + d_k gt_jl - d_j gt_kl) / 2
    G = np.zeros((3,) + gti.shape[1:])
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    gl = 0.5 * (dg[l][SYM[(j, k)]] + dg[k][SYM[(j, l)]]
                                - dg[j][SYM[(k, l)]])
                    G[i] += gtu[i, j] * gtu[k, l] * gl
    v[GAMX:GAMX + 3, gc:-gc, gc:-gc, gc:-gc] = G
    extrapolate_layers(grid, v[GAMX:GAMX + 3])
    return out


# ---- puncture tracking ----------------------------------------------------
# It follows the object-tracking subsection of the paper's analysis
# section: a puncture moves with dx^i/dt = -beta^i, the shift interpolated
# to its position, integrated with one first-order Euler step per call.
# Reading: the interpolation is tricubic Lagrange on the 4 x 4 x 4 storage
# points around the position (base node floor((x - x_0)/h) - 1 per axis,
# x_0 the coordinate of storage index 0), the block shifted inward where it
# would leave the storage grid.
def lagrange4(t):
    """Weights of the cubic through nodes 0, 1, 2, 3 at parameter t."""
    w = []
    for m in range(4):
        p = 1.0
        for l in range(4):
            if l != m:
                p *= (t - l) / (m - l)
        w.append(p)
    return w


def shift_at(grid, u, pos):
    """beta^i at each position (array (n, 3)) by tricubic interpolation."""
    v = grid.view(u)
    out = []
    for x in np.asarray(pos, float):
        base, wts = [], []
        for a in range(3):
            N = grid.n[a] + 2 * grid.ghost
            x0 = grid.origin[a] - grid.ghost * grid.h[a]
            s = (x[a] - x0) / grid.h[a]
            b = int(np.floor(s)) - 1
            b = min(max(b, 0), N - 4)
            base.append(b)
            wts.append(lagrange4(s - b))
        beta = []
        for c in range(3):
            f = v[BETX + c]
            acc = 0.0
            for k in range(4):
                for j in range(4):
                    for i in range(4):
                        acc += (wts[2][k] * wts[1][j] * wts[0][i] *
                                f[base[2] + k, base[1] + j, base[0] + i])
            beta.append(acc)
        out.append(beta)
    return np.array(out)


def track_punctures(grid, u, pos, dt):
    """One Euler step of dx/dt = -beta(x) for every position."""
    return np.asarray(pos, float) - dt * shift_at(grid, u, pos)
