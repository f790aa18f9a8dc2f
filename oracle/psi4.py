"""Oracle for the Weyl scalar Psi_4 (test infrastructure: only tests/, the
smoke check and the benchmark's CPU baseline use it).

Follows the paper's Analysis section, "Gravitational Waves" (WeylScal4):
Psi_4 = C_abcd n^a mbar^b n^c mbar^d, the Weyl tensor (the Riemann tensor in
vacuum) projected onto the fiducial null tetrad
    l = (u + r)/sqrt2,  n = (u - r)/sqrt2,  m = (theta + i phi)/sqrt2,
u the unit normal of the slice; the spatial triad starts from
    phi~ = (-y, x, 0),  r~ = (x, y, z),
    theta~^i = sqrt(det gamma) gamma^ik eps_klm phi~^l r~^m
and is made orthonormal with the 3-metric by Gram-Schmidt, phi~ normalised
first (then r against phi, then theta against phi and r).  Psi_4 is
evaluated in the printed 3+1 form
    Psi_4 = R_ijkl n^i mb^j n^k mb^l
          + 2 R_0jkl (n^0 mb^j n^k mb^l - mb^0 n^j n^k mb^l)
          + R_0j0l (n^0 mb^j n^0 mb^l + mb^0 n^j mb^0 n^l
                    - 2 n^0 mb^j mb^0 n^l)
with the index 0 the projection on u (so n^0 = 1/sqrt2 and, for this
tetrad, mb^0 = 0), the space-time Riemann components from the 3+1 data by
the vacuum Gauss, Codazzi and Ricci equations (K_ij = -(1/2) L_u gamma_ij,
the sign of d_t gamma_ij = -2 alpha K_ij + ...):
    R_ijkl = 3R_ijkl + K_ik K_jl - K_il K_jk,
    R_0jkl = D_k K_jl - D_l K_jk,
    R_0j0l = 3R_jl + K K_jl - K_jm K^m_l.

Discretisation (a reading: the paper evaluates Psi_4 from the metric and
its derivatives without fixing a scheme): the ADM variables are formed from the BSSN state pointwise
by inverting the paper's definitions, gamma_ij = e^{4 phi} gt_ij and
K_ij = e^{4 phi} (At_ij + gt_ij K / 3), at every storage point; at interior
points gamma_ij is differenced with the evolution's centred stencils (first,
pure second and mixed = tensor product of first derivatives) and K_ij with
the centred first-derivative stencil; the rest is pointwise algebra
(psi4_point), in FP64.  Coordinates x^i of the tetrad are measured from a
given centre (default the origin).
"""
import numpy as np

# centred stencil weights on u(+k) - u(-k) (first) and u(+k) + u(-k) - 2 u(0)
# (second), k = 1.., exact on polynomials of degree <= order
_A = {4: (2 / 3, -1 / 12), 8: (4 / 5, -1 / 5, 4 / 105, -1 / 280)}
_B = {4: (4 / 3, -1 / 12), 8: (8 / 5, -1 / 5, 8 / 315, -1 / 560)}

SYM = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
PHI, GXX, TRK, AXX = 0, 1, 7, 8


def _sym(a6):
    """[6, ...] symmetric components -> [3, 3, ...]."""
    m = [[None] * 3 for _ in range(3)]
    for c, (i, j) in enumerate(SYM):
        m[i][j] = m[j][i] = a6[c]
    return np.array(m)


def adm_from_state(grid, u):
    """gamma_ij and K_ij ([3, 3, z, y, x] over the storage grid) from the
    BSSN state by the paper's definitions inverted."""
    v = grid.view(u)
    e4 = np.exp(4.0 * v[PHI])
    gt = _sym([v[GXX + c] for c in range(6)])
    At = _sym([v[AXX + c] for c in range(6)])
    gam = e4 * gt
    K = e4 * (At + gt * v[TRK] / 3.0)
    return gam, K


def _shift(f, grid, off):
    """Interior window of storage array f ([..., z, y, x]) shifted by the
    integer offsets off = (dx, dy, dz)."""
    g = grid.ghost
    n = grid.n
    return f[..., g + off[2]:g + off[2] + n[2], g + off[1]:g + off[1] + n[1],
             g + off[0]:g + off[0] + n[0]]


def _unit(a, k):
    o = [0, 0, 0]
    o[a] = k
    return o


def derivatives(grid, f, order, second=True):
    """Centred differences of f at interior points: d[a] = d_a f and, with
    second, dd[a][b] = d_a d_b f (pure: second-derivative stencil; mixed:
    the tensor product of first-derivative stencils)."""
    A, Bw = _A[order], _B[order]
    h = grid.h
    f0 = _shift(f, grid, (0, 0, 0))
    d = []
    for a in range(3):
        s = 0.0
        for k, w in enumerate(A, start=1):
            s = s + w * (_shift(f, grid, _unit(a, k)) -
                         _shift(f, grid, _unit(a, -k)))
        d.append(s / h[a])
    if not second:
        return np.array(d), None
    dd = [[None] * 3 for _ in range(3)]
    for a in range(3):
        s = 0.0
        for k, w in enumerate(Bw, start=1):
            s = s + w * (_shift(f, grid, _unit(a, k)) +
                         _shift(f, grid, _unit(a, -k)) - 2.0 * f0)
        dd[a][a] = s / (h[a] * h[a])
        for b in range(a + 1, 3):
            s = 0.0
            for i, wi in enumerate(A, start=1):
                for j, wj in enumerate(A, start=1):
                    def at(si, sj):
                        o = [0, 0, 0]
                        o[a] += si * i
                        o[b] += sj * j
                        return _shift(f, grid, o)
                    s = s + wi * wj * (at(1, 1) - at(1, -1) - at(-1, 1) +
                                       at(-1, -1))
            dd[a][b] = dd[b][a] = s / (h[a] * h[b])
    return np.array(d), np.array(dd)


def tetrad(gam, x):
    """Orthonormal spatial triad (rhat, thetahat, phihat) of the fiducial
    tetrad at points x ([3, ...]) for the 3-metric gam ([3, 3, ...])."""
    ginv = np.linalg.inv(np.moveaxis(gam, (0, 1), (-2, -1)))
    ginv = np.moveaxis(ginv, (-2, -1), (0, 1))
    sdet = np.sqrt(np.linalg.det(np.moveaxis(gam, (0, 1), (-2, -1))))

    def dot(a, b):
        return np.einsum("i...,ij...,j...->...", a, gam, b)

    zero = np.zeros_like(x[0])
    phi = np.array([-x[1], x[0], zero])
    r = np.array(x, dtype=float)
    eps = np.zeros((3, 3, 3))
    eps[0, 1, 2] = eps[1, 2, 0] = eps[2, 0, 1] = 1.0
    eps[0, 2, 1] = eps[2, 1, 0] = eps[1, 0, 2] = -1.0
    th = sdet * np.einsum("ik...,klm,l...,m...->i...", ginv, eps, phi, r)
    # Gram-Schmidt: phi first, then r, then theta
    phi = phi / np.sqrt(dot(phi, phi))
    r = r - dot(r, phi) * phi
    r = r / np.sqrt(dot(r, r))
    th = th - dot(th, phi) * phi - dot(th, r) * r
    th = th / np.sqrt(dot(th, th))
    return r, th, phi


def psi4_point(gam, dgam, ddgam, K, dK, x):
    """Psi_4 (complex) from the 3-metric gam[i,j], its derivatives
    dgam[k,i,j] = d_k gamma_ij and ddgam[k,l,i,j] = d_k d_l gamma_ij, the
    extrinsic curvature K[i,j] and dK[k,i,j] = d_k K_ij, at coordinates x
    (relative to the tetrad's centre); trailing axes are points."""
    ginv = np.linalg.inv(np.moveaxis(gam, (0, 1), (-2, -1)))
    ginv = np.moveaxis(ginv, (-2, -1), (0, 1))
    # Christoffels, first index lowered: G_kij = (d_i g_kj + d_j g_ki - d_k g_ij)/2
    Gl = 0.5 * (np.einsum("ikj...->kij...", dgam) +
                np.einsum("jki...->kij...", dgam) - dgam)
    Gu = np.einsum("mk...,kij...->mij...", ginv, Gl)
    # 3-Riemann, all indices down:
    # R_ijkl = (d_j d_k g_il + d_i d_l g_jk - d_i d_k g_jl - d_j d_l g_ik)/2
    #          + g_mn (G^m_jk G^n_il - G^m_jl G^n_ik)
    R = 0.5 * (np.einsum("jkil...->ijkl...", ddgam) +
               np.einsum("iljk...->ijkl...", ddgam) -
               np.einsum("ikjl...->ijkl...", ddgam) -
               np.einsum("jlik...->ijkl...", ddgam))
    R = R + np.einsum("mn...,mjk...,nil...->ijkl...", gam, Gu, Gu) \
        - np.einsum("mn...,mjl...,nik...->ijkl...", gam, Gu, Gu)
    Ric = np.einsum("ik...,ijkl...->jl...", ginv, R)
    trK = np.einsum("ij...,ij...->...", ginv, K)
    Kud = np.einsum("mk...,kl...->ml...", ginv, K)  # K^m_l
    # D_k K_ij = d_k K_ij - G^m_ki K_mj - G^m_kj K_im
    DK = dK - np.einsum("mki...,mj...->kij...", Gu, K) \
        - np.einsum("mkj...,im...->kij...", Gu, K)
    # space-time Riemann projections (vacuum Gauss, Codazzi, Ricci)
    R4 = R + np.einsum("ik...,jl...->ijkl...", K, K) \
        - np.einsum("il...,jk...->ijkl...", K, K)
    R0 = np.einsum("kjl...->jkl...", DK) - np.einsum("ljk...->jkl...", DK)
    E = Ric + trK * K - np.einsum("jm...,ml...->jl...", K, Kud)
    # tetrad
    rh, th, ph = tetrad(gam, x)
    s2 = np.sqrt(0.5)
    n0 = s2
    nv = -s2 * rh
    mb0 = 0.0
    mbv = s2 * (th - 1j * ph)
    t1 = np.einsum("ijkl...,i...,j...,k...,l...->...", R4, nv, mbv, nv, mbv)
    t2 = 2.0 * (n0 * np.einsum("jkl...,j...,k...,l...->...", R0, mbv, nv,
                               mbv) -
                mb0 * np.einsum("jkl...,j...,k...,l...->...", R0, nv, nv,
                                mbv))
    t3 = (n0 * n0 * np.einsum("jl...,j...,l...->...", E, mbv, mbv)
          + mb0 * mb0 * np.einsum("jl...,j...,l...->...", E, nv, nv)
          - 2.0 * n0 * mb0 * np.einsum("jl...,j...,l...->...", E, mbv, nv))
    return t1 + t2 + t3


def psi4(grid, order, u, centre=(0.0, 0.0, 0.0)):
    """Psi_4 at every interior point ([z, y, x] complex array) of the BSSN
    state u (flat buffer in the grid's layout)."""
    gam, K = adm_from_state(grid, u)
    dg = np.zeros((3, 3, 3) + tuple(grid.n[::-1]))
    ddg = np.zeros((3, 3, 3, 3) + tuple(grid.n[::-1]))
    dK = np.zeros((3, 3, 3) + tuple(grid.n[::-1]))
    for i, j in SYM:
        d, dd = derivatives(grid, gam[i, j], order)
        dg[:, i, j] = dg[:, j, i] = d
        ddg[:, :, i, j] = ddg[:, :, j, i] = dd
        d, _ = derivatives(grid, K[i, j], order, second=False)
        dK[:, i, j] = dK[:, j, i] = d
    g0 = _shift(gam, grid, (0, 0, 0))
    K0 = _shift(K, grid, (0, 0, 0))
    nz, ny, nx = grid.n[2], grid.n[1], grid.n[0]
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                             indexing="ij")
    x = np.array([grid.origin[0] + xx * grid.h[0] - centre[0],
                  grid.origin[1] + yy * grid.h[1] - centre[1],
                  grid.origin[2] + zz * grid.h[2] - centre[2]])
    return psi4_point(g0, dg, ddg, K0, dK, x)
