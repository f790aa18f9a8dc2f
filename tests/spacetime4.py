"""Exact vacuum space-times as 4-metrics, for pinning the Psi_4 oracle
(test-only; shares nothing with oracle/psi4.py).

A space-time is given by sympy expressions of its 4-metric g_{mu nu}(t, x,
y, z), its inverse, and (where sympy would be slow) the inverse 3-metric and
the lapse in closed form.  Everything else is derived here by a route that
never uses the 3+1 split of the Riemann tensor:

  * the 4-Riemann tensor from the Christoffel symbols of g by the
    definition R^r_{s m n} = d_m G^r_{n s} - d_n G^r_{m s}
    + G^r_{m l} G^l_{n s} - G^r_{n l} G^l_{m s}, differentiated by sympy;
  * the 3+1 data at fixed t: gamma_ij = g_ij, beta_i = g_0i,
    beta^i = gamma^ij beta_j, alpha^2 = beta^i beta_i - g_00, and
    K_ij = -(d_t gamma_ij - D_i beta_j - D_j beta_i) / (2 alpha), with sympy
    derivatives of gamma and K for the stencil-free inputs of psi4_point;
  * the unit normal u^mu = (1, -beta^i) / alpha.

Space-times: a plane-fronted gravitational wave (pp-wave) in Kerr-Schild
form g = eta + H k k with k = dt - dz and H harmonic in (x, y), an exact
vacuum solution for any profile along u = t - z; and Schwarzschild in
Kerr-Schild coordinates, g = eta + 2 M/r l l, centred anywhere.
"""
import numpy as np

sp = None


def _sympy():
    global sp
    if sp is None:
        import sympy
        sp = sympy
    return sp


class Spacetime:
    def __init__(self, g, ginv, gami=None, alp=None):
        s = _sympy()
        t, x, y, z = s.symbols("t x y z", real=True)
        self.X4 = X4 = (t, x, y, z)
        self.g, self.ginv = g, ginv
        n = 4
        dg = [[[s.diff(g[a, b], X4[c]) for c in range(n)] for b in range(n)]
              for a in range(n)]
        G = [[[sum(ginv[r, q] * (dg[q][m][v] + dg[q][v][m] - dg[m][v][q])
                   for q in range(n)) / 2 for v in range(n)]
              for m in range(n)] for r in range(n)]
        dG = [[[[s.diff(G[r][m][q], X4[k]) for k in range(n)]
                for q in range(n)] for m in range(n)] for r in range(n)]
        lam = lambda e: s.lambdify(
            X4, e.tolist() if hasattr(e, "tolist") else e, "numpy", cse=True)
        self._G = lam(s.Array(G))
        self._dG = lam(s.Array(dG))
        self._g = lam(g)
        # 3+1 data
        gam = g[1:, 1:]
        bl = s.Matrix([g[0, i] for i in range(1, 4)])
        gami = gam.inv() if gami is None else gami
        bu = gami * bl
        if alp is None:
            alp = s.sqrt((bl.T * bu)[0] - g[0, 0])
        X3 = X4[1:]
        G3 = [[[sum(gami[k, l] * (s.diff(gam[l, i], X3[j]) +
                                  s.diff(gam[l, j], X3[i]) -
                                  s.diff(gam[i, j], X3[l]))
                    for l in range(3)) / 2 for j in range(3)]
               for i in range(3)] for k in range(3)]
        K = s.Matrix(3, 3, lambda i, j: -(
            s.diff(gam[i, j], t) - s.diff(bl[j], X3[i]) -
            s.diff(bl[i], X3[j]) +
            2 * sum(G3[k][i][j] * bl[k] for k in range(3))) / (2 * alp))
        self._gam = lam(gam)
        self._dgam = lam(s.Array([[[s.diff(gam[i, j], X3[k])
                                    for j in range(3)] for i in range(3)]
                                  for k in range(3)]))
        self._ddgam = lam(s.Array([[[[s.diff(gam[i, j], X3[k], X3[l])
                                      for j in range(3)] for i in range(3)]
                                    for l in range(3)] for k in range(3)]))
        self._K = lam(K)
        self._dK = lam(s.Array([[[s.diff(K[i, j], X3[k]) for j in range(3)]
                                 for i in range(3)] for k in range(3)]))
        self._alp = lam(alp)
        self._bu = lam(bu)

    def riemann_down(self, p):
        """R_{a b c d} (all indices down) at the event p = (t, x, y, z)."""
        G = np.array(self._G(*p), float)
        D = np.array(self._dG(*p), float)  # D[r, m, s, k] = d_k G^r_{m s}
        R = (np.einsum("rnsm->rsmn", D) - np.einsum("rmsn->rsmn", D)
             + np.einsum("rml,lns->rsmn", G, G)
             - np.einsum("rnl,lms->rsmn", G, G))
        return np.einsum("ar,rsmn->asmn", np.array(self._g(*p), float), R)

    def metric(self, p):
        return np.array(self._g(*p), float)

    def adm(self, p):
        """(gamma[i,j], dgamma[k,i,j], ddgamma[k,l,i,j], K[i,j], dK[k,i,j],
        alpha, beta^i) at p."""
        f = lambda fn: np.array(fn(*p), float)
        return (f(self._gam), f(self._dgam), f(self._ddgam), f(self._K),
                f(self._dK), float(self._alp(*p)), f(self._bu).ravel())

    def adm_arrays(self, t, X, Y, Z):
        """(gamma, dgamma, ddgamma, K, dK) as in adm, on arrays of points
        (trailing axes)."""
        T = np.full_like(X, t)

        def arr(nested):
            if hasattr(nested, "tolist") and getattr(nested, "ndim", 0) and \
                    nested.dtype == object:
                nested = nested.tolist()
            if isinstance(nested, (list, tuple)):
                return np.stack([arr(e) for e in nested])
            return np.broadcast_to(np.asarray(nested, float), X.shape)

        return tuple(arr(fn(T, X, Y, Z)) for fn in (self._gam, self._dgam, self._ddgam, self._K,
                                self._dK))

    def adm_fields(self, t, X, Y, Z):
        """gamma_ij and K_ij on arrays of points (values only)."""
        gam, _, _, K, _ = self.adm_arrays(t, X, Y, Z)
        return gam, K


def pp_wave(amp=(0.3, 0.2), omega=(1.0, 2.0)):
    """H = a0 sin(w0 u) (x^2 - y^2) + a1 cos(w1 u) x y, u = t - z."""
    s = _sympy()
    t, x, y, z = s.symbols("t x y z", real=True)
    u = t - z
    H = (s.nsimplify(amp[0]) * s.sin(s.nsimplify(omega[0]) * u) * (x**2 - y**2)
         + s.nsimplify(amp[1]) * s.cos(s.nsimplify(omega[1]) * u) * x * y)
    k = s.Matrix([1, 0, 0, -1])
    eta = s.diag(-1, 1, 1, 1)
    ku = eta * k
    return Spacetime(eta + H * k * k.T, eta - H * ku * ku.T)


def schwarzschild_ks(M=1, centre=(0, 0, 0)):
    s = _sympy()
    t, x, y, z = s.symbols("t x y z", real=True)
    c = [s.nsimplify(v) for v in centre]
    M = s.nsimplify(M)
    r = s.sqrt((x - c[0])**2 + (y - c[1])**2 + (z - c[2])**2)
    l = s.Matrix([1, (x - c[0]) / r, (y - c[1]) / r, (z - c[2]) / r])
    H = M / r
    eta = s.diag(-1, 1, 1, 1)
    lu = eta * l
    L3 = l[1:, :]
    gami = s.eye(3) - 2 * H / (1 + 2 * H) * L3 * L3.T
    return Spacetime(eta + 2 * H * l * l.T, eta - 2 * H * lu * lu.T,
                     gami=gami, alp=1 / s.sqrt(1 + 2 * H))


def psi4_4d(st, p, triad):
    """Psi_4 = R_abcd n^a mb^b n^c mb^d from the 4-Riemann tensor, with
    n = (u - rhat)/sqrt2 and mb = (thetahat - i phihat)/sqrt2 as 4-vectors
    (rhat, thetahat, phihat = the spatial triad at p)."""
    R = st.riemann_down(p)
    _, _, _, _, _, alp, bu = st.adm(p)
    rh, th, ph = triad
    u = np.r_[1.0 / alp, -bu / alp]
    n = (u - np.r_[0.0, rh]) / np.sqrt(2.0)
    mb = np.r_[0.0, th - 1j * ph] / np.sqrt(2.0)
    return np.einsum("abcd,a,b,c,d->", R, n, mb, n, mb)
