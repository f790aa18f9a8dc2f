/*
 * bssn_oracle.c -- plain, slow, FP64 CPU reference of the vacuum BSSN
 * right-hand side, the classical RK4 step and the ADM constraints.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or helper with the HIP library: its structs, slot numbering
 * and stencil weights are written out again here on purpose.
 *
 * What it follows (Einstein Toolkit paper, arXiv:1111.3344):
 *   - BSSN variables and their definitions: section "Spacetime Curvature
 *     Evolution", definition equations of phi, gamma~, K, A~, Gamma~.
 *   - Evolution equations for alpha, K, beta, B, phi, gamma~, A~, Gamma~ with
 *     m = 1, the partial_0 = partial_t - beta^j partial_j convention, and the
 *     Ricci split R~_ij + R^phi_ij: same section, evolution and Ricci
 *     equations.
 *   - 1+log slicing f = 2/alpha, K_0 = 0; Gamma-driver G = 3/(4 alpha^2),
 *     H = exp(4 phi), eta = B q(r)/2, q(r) = 1 (r <= R), R/r (r >= R): same
 *     section, gauge equations and the attenuation equation.
 *   - Fourth-order centred finite differences and fifth-order Kreiss-Oliger
 *     dissipation: same section, opening paragraph.  Eighth-order variant:
 *     "Conclusion and Future Work" (eighth-order convergence of BH codes).
 *   - Method-of-lines separation of RHS and time integration: "HydroBase"
 *     schedule groups and the GRHydro method-of-lines remark.
 *   - Constraints H = R - K^i_j K^j_i + K^2, M_i = D_j K_i^j - D_i K:
 *     section "Other analysis modules".
 *
 * Readings where the paper is silent (each is repeated where it is used):
 *   - classical RK4 (c = 0,1/2,1/2,1; b = 1/6,1/3,1/3,1/6);
 *   - advection by the lopsided (upwind) stencil on the side of sign(beta);
 *   - KO operator  +eps (-1)^(r+1) h^(2r-1) 2^(-2r) (D+D-)^r, r = 3 (4th
 *     order) or 5 (8th order), on every slot and every axis;
 *   - derivatives of the inverse conformal metric by the identity
 *     d_k g^ij = -g^ia g^jb d_k g_ab, never by differencing g^ij;
 *   - the evolved Gamma~^i enters only through d_j Gamma~^k in R~_ij; every
 *     other Gamma~ in the equations is  Gd^i = sum_l d_l g^li;
 *   - vacuum: all matter terms dropped;
 *   - slot 24 ("A", the lapse time-derivative variable) has zero source and
 *     is only advected and dissipated;
 *   - every stencil is evaluated on differences taken from the centre value
 *     (first derivatives on the pairwise differences u(+k)-u(-k)).
 *
 * Parity pins: see the test suite (Minkowski zero, polynomial exactness,
 * stationary Kerr-Schild, Brill-Lindquist closed forms, Kasner, RK4
 * stability polynomial, KO checkerboard, constraint convergence).
 *
 * Compiled with -O2 -fopenmp -ffp-contract=off -fno-fast-math.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- the oracle's own description of a grid and of the parameters ------- */
typedef struct {
  int32_t n[3];        /* interior points along x, y, z                     */
  int32_t ghost;       /* ghost layers on every face                        */
  int64_t sy, sz, sf;  /* element strides of a y-row, a z-plane and a slot  */
  double origin[3];    /* coordinate of interior point (0,0,0)              */
  double h[3];         /* grid spacing                                       */
  int32_t bc;          /* 0 static ghosts, 1 periodic                        */
} oracle_grid;

typedef struct {
  int32_t fd_order;    /* 4 or 8                                             */
  double ko_eps;       /* Kreiss-Oliger strength                             */
  double lapse_f;      /* f = lapse_f / alpha                                */
  double shift_G;      /* G = shift_G / alpha^2                              */
  double eta;          /* eta^i = eta * q(r) * B^i                           */
  double eta_R;        /* transition radius of q(r); <= 0 or inf: q = 1      */
  int32_t lapse_static, shift_static;
} oracle_params;

/* slot numbering of the 25 evolved grid functions */
enum {
  S_PHI = 0, S_GXX = 1, S_GXY, S_GXZ, S_GYY, S_GYZ, S_GZZ, S_K = 7,
  S_AXX = 8, S_AXY, S_AXZ, S_AYY, S_AYZ, S_AZZ, S_GAMX = 14, S_GAMY, S_GAMZ,
  S_ALP = 17, S_BETX = 18, S_BETY, S_BETZ, S_BX = 21, S_BY, S_BZ, S_ADOT = 24,
  NSLOT = 25
};

/* symmetric 3x3 index pair -> position 0..5 (xx xy xz yy yz zz) */
static int sym6(int i, int j) {
  static const int t[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
  return t[i][j];
}

/* ---- reading the state ---------------------------------------------------
 * Interior indices run 0..n-1; a stencil may reach ghost+... outside.  For a
 * periodic grid the index wraps modulo n (ghost memory is never read); for a
 * static grid the ghost memory holds the boundary data. */
static int wrap(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

static double U(const oracle_grid* g, const double* u, int f, int i, int j,
                int k) {
  if (g->bc == 1) {
    i = wrap(i, g->n[0]);
    j = wrap(j, g->n[1]);
    k = wrap(k, g->n[2]);
  }
  int64_t gh = g->ghost;
  return u[(int64_t)f * g->sf + (k + gh) * g->sz + (j + gh) * g->sy + (i + gh)];
}

static int64_t IDX(const oracle_grid* g, int f, int i, int j, int k) {
  int64_t gh = g->ghost;
  return (int64_t)f * g->sf + (k + gh) * g->sz + (j + gh) * g->sy + (i + gh);
}

/* value of slot f at (p + a*e_axis + b*e_axis2) */
static double U2(const oracle_grid* g, const double* u, int f, const int p[3],
                 int ax, int a, int ax2, int b) {
  int q[3] = {p[0], p[1], p[2]};
  q[ax] += a;
  q[ax2] += b;
  return U(g, u, f, q[0], q[1], q[2]);
}

static double U1(const oracle_grid* g, const double* u, int f, const int p[3],
                 int ax, int a) {
  int q[3] = {p[0], p[1], p[2]};
  q[ax] += a;
  return U(g, u, f, q[0], q[1], q[2]);
}

/* ---- finite-difference operators ----------------------------------------
 * Weights are the unique ones that are exact on polynomials of the highest
 * degree their point set allows (centred 5/9-point first and second
 * derivatives, lopsided 5/9-point first derivatives) and the binomial
 * (D+D-)^r for Kreiss-Oliger. */

/* centred first derivative: sum_k a_k (u(+k) - u(-k)) / h */
static double d1(const oracle_grid* g, const double* u, int f, const int p[3],
                 int ax, int order) {
  static const double a4[2] = {2.0 / 3.0, -1.0 / 12.0};
  static const double a8[4] = {4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0,
                               -1.0 / 280.0};
  const double* a = order == 8 ? a8 : a4;
  int m = order == 8 ? 4 : 2;
  double s = 0.0;
  for (int k = 1; k <= m; ++k)
    s += a[k - 1] * (U1(g, u, f, p, ax, k) - U1(g, u, f, p, ax, -k));
  return s / g->h[ax];
}

/* centred second derivative: sum_{k != 0} b_k (u(k) - u(0)) / h^2 */
static double d2(const oracle_grid* g, const double* u, int f, const int p[3],
                 int ax, int order) {
  static const double b4[2] = {4.0 / 3.0, -1.0 / 12.0};
  static const double b8[4] = {8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0,
                               -1.0 / 560.0};
  const double* b = order == 8 ? b8 : b4;
  int m = order == 8 ? 4 : 2;
  double u0 = U(g, u, f, p[0], p[1], p[2]);
  double s = 0.0;
  for (int k = 1; k <= m; ++k)
    s += b[k - 1] * ((U1(g, u, f, p, ax, k) - u0) +
                     (U1(g, u, f, p, ax, -k) - u0));
  return s / (g->h[ax] * g->h[ax]);
}

/* mixed second derivative d_ax d_ax2: the tensor product of two centred
 * first-derivative stencils, sum_{a,b} w_a w_b (u(a,b) - u(0,0)). */
static double d11(const oracle_grid* g, const double* u, int f,
                  const int p[3], int ax, int ax2, int order) {
  static const double w4[5] = {1.0 / 12.0, -2.0 / 3.0, 0.0, 2.0 / 3.0,
                               -1.0 / 12.0};
  static const double w8[9] = {1.0 / 280.0, -4.0 / 105.0, 1.0 / 5.0,
                               -4.0 / 5.0,  0.0,          4.0 / 5.0,
                               -1.0 / 5.0,  4.0 / 105.0,  -1.0 / 280.0};
  const double* w = order == 8 ? w8 : w4;
  int m = order == 8 ? 4 : 2;
  double u0 = U(g, u, f, p[0], p[1], p[2]);
  double s = 0.0;
  for (int a = -m; a <= m; ++a) {
    if (a == 0) continue;
    for (int b = -m; b <= m; ++b) {
      if (b == 0) continue;
      s += w[a + m] * w[b + m] * (U2(g, u, f, p, ax, a, ax2, b) - u0);
    }
  }
  return s / (g->h[ax] * g->h[ax2]);
}

/* lopsided first derivative on the side of sign(beta):
 * beta > 0 uses offsets -1..3 (4th) / -3..5 (8th); beta < 0 the mirror. */
static double dup(const oracle_grid* g, const double* u, int f,
                  const int p[3], int ax, double beta, int order) {
  static const double p4[5] = {-3.0 / 12.0, -10.0 / 12.0, 18.0 / 12.0,
                               -6.0 / 12.0, 1.0 / 12.0}; /* k = -1..3 */
  static const double p8[9] = {-1.0 / 168.0, 1.0 / 14.0, -1.0 / 2.0,
                               -9.0 / 20.0,  5.0 / 4.0,  -1.0 / 2.0,
                               1.0 / 6.0,    -1.0 / 28.0, 1.0 / 280.0};
  /* k = -3..5 */
  const double* w = order == 8 ? p8 : p4;
  int lo = order == 8 ? -3 : -1;
  int npt = order == 8 ? 9 : 5;
  double u0 = U(g, u, f, p[0], p[1], p[2]);
  double s = 0.0;
  if (beta > 0.0) {
    for (int t = 0; t < npt; ++t) {
      int k = lo + t;
      if (k == 0) continue;
      s += w[t] * (U1(g, u, f, p, ax, k) - u0);
    }
  } else if (beta < 0.0) {
    /* mirror image: weight at offset -k is minus the weight at +k */
    for (int t = 0; t < npt; ++t) {
      int k = lo + t;
      if (k == 0) continue;
      s += -w[t] * (U1(g, u, f, p, ax, -k) - u0);
    }
  } else {
    return 0.0; /* only ever multiplied by beta = 0 */
  }
  return s / g->h[ax];
}

/* Kreiss-Oliger term along one axis, already with its sign and scaling:
 * eps (-1)^(r+1) h^(2r-1) 2^(-2r) (D+D-)^r u, r = 3 or 5. */
static double ko(const oracle_grid* g, const double* u, int f, const int p[3],
                 int ax, double eps, int order) {
  static const double c3[4] = {-20.0, 15.0, -6.0, 1.0};   /* (D+D-)^3 h^6 */
  static const double c5[6] = {-252.0, 210.0, -120.0, 45.0, -10.0, 1.0};
  int r = order == 8 ? 5 : 3;
  const double* c = order == 8 ? c5 : c3;
  double u0 = U(g, u, f, p[0], p[1], p[2]);
  double s = 0.0; /* sum of weights is 0, so use centre differences */
  for (int k = 1; k <= r; ++k)
    s += c[k] * ((U1(g, u, f, p, ax, k) - u0) + (U1(g, u, f, p, ax, -k) - u0));
  double sign = (r + 1) % 2 == 0 ? 1.0 : -1.0;
  double scale = ldexp(1.0, -2 * r); /* 2^-2r */
  /* h^(2r-1) (D+D-)^r = h^(-1) * (h^(2r) (D+D-)^r) */
  return sign * eps * scale * s / g->h[ax];
}

/* ---- the pointwise right-hand side ---------------------------------------
 * Evaluates every equation at interior point p and writes 25 values. */
static void rhs_point(const oracle_grid* g, const oracle_params* P,
                      const double* u, const int p[3], double out[NSLOT]) {
  const int ord = P->fd_order;
  double v[NSLOT];
  for (int f = 0; f < NSLOT; ++f) v[f] = U(g, u, f, p[0], p[1], p[2]);

  /* conformal metric, its inverse through the adjugate, A~ */
  double gt[3][3], At[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      gt[i][j] = v[S_GXX + sym6(i, j)];
      At[i][j] = v[S_AXX + sym6(i, j)];
    }
  double det = gt[0][0] * (gt[1][1] * gt[2][2] - gt[1][2] * gt[2][1]) -
               gt[0][1] * (gt[1][0] * gt[2][2] - gt[1][2] * gt[2][0]) +
               gt[0][2] * (gt[1][0] * gt[2][1] - gt[1][1] * gt[2][0]);
  double gu[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      /* adjugate: transpose of the cofactor matrix */
      int r0 = (j + 1) % 3, r1 = (j + 2) % 3, c0 = (i + 1) % 3,
          c1 = (i + 2) % 3;
      gu[i][j] = (gt[r0][c0] * gt[r1][c1] - gt[r0][c1] * gt[r1][c0]) / det;
    }

  const double phi = v[S_PHI], trK = v[S_K], alpha = v[S_ALP];
  double beta[3] = {v[S_BETX], v[S_BETY], v[S_BETZ]};
  double Bv[3] = {v[S_BX], v[S_BY], v[S_BZ]};

  /* first derivatives */
  double dgt[3][3][3]; /* dgt[i][j][k] = d_k gt_ij */
  double dphi[3], dalp[3], dK[3], dbeta[3][3] /* [i][j] = d_j beta^i */,
      dGam[3][3] /* [k][j] = d_j Gamma~^k */;
  for (int k = 0; k < 3; ++k) {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        dgt[i][j][k] = d1(g, u, S_GXX + sym6(i, j), p, k, ord);
    dphi[k] = d1(g, u, S_PHI, p, k, ord);
    dalp[k] = d1(g, u, S_ALP, p, k, ord);
    dK[k] = d1(g, u, S_K, p, k, ord);
    for (int i = 0; i < 3; ++i) {
      dbeta[i][k] = d1(g, u, S_BETX + i, p, k, ord);
      dGam[i][k] = d1(g, u, S_GAMX + i, p, k, ord);
    }
  }
  /* second derivatives: pure on the diagonal, tensor product off it */
  double ddgt[3][3][3][3], ddphi[3][3], ddalp[3][3], ddbeta[3][3][3];
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l) {
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          ddgt[i][j][k][l] =
              k == l ? d2(g, u, S_GXX + sym6(i, j), p, k, ord)
                     : d11(g, u, S_GXX + sym6(i, j), p, k, l, ord);
      ddphi[k][l] = k == l ? d2(g, u, S_PHI, p, k, ord)
                           : d11(g, u, S_PHI, p, k, l, ord);
      ddalp[k][l] = k == l ? d2(g, u, S_ALP, p, k, ord)
                           : d11(g, u, S_ALP, p, k, l, ord);
      for (int i = 0; i < 3; ++i)
        ddbeta[i][k][l] = k == l ? d2(g, u, S_BETX + i, p, k, ord)
                                 : d11(g, u, S_BETX + i, p, k, l, ord);
    }

  /* Christoffel symbols of gt: first kind Gl[i][j][k] = Gamma~_ijk (first
   * index lowered), second kind Gu[i][j][k] = Gamma~^i_jk */
  double Gl[3][3][3], Gu[3][3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k)
        Gl[i][j][k] = 0.5 * (dgt[i][j][k] + dgt[i][k][j] - dgt[j][k][i]);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) {
        double s = 0.0;
        for (int l = 0; l < 3; ++l) s += gu[i][l] * Gl[l][j][k];
        Gu[i][j][k] = s;
      }
  /* derivative of the inverse metric by the identity, and Gd^i */
  double dgu[3][3][3]; /* dgu[i][j][k] = d_k gu^ij */
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) {
        double s = 0.0;
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) s -= gu[i][a] * gu[j][b] * dgt[a][b][k];
        dgu[i][j][k] = s;
      }
  double Gd[3];
  for (int i = 0; i < 3; ++i) {
    double s = 0.0;
    for (int l = 0; l < 3; ++l) s += dgu[l][i][l];
    Gd[i] = s;
  }

  /* conformal Ricci tensor R~_ij */
  double Rt[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) s += -0.5 * gu[k][l] * ddgt[i][j][k][l];
      for (int k = 0; k < 3; ++k)
        s += 0.5 * (gt[k][i] * dGam[k][j] + gt[k][j] * dGam[k][i]);
      for (int k = 0; k < 3; ++k)
        s += -0.5 * (Gl[i][j][k] + Gl[j][i][k]) * Gd[k];
      for (int l = 0; l < 3; ++l)
        for (int m = 0; m < 3; ++m)
          for (int k = 0; k < 3; ++k)
            s += gu[l][m] * (Gu[k][l][i] * Gl[j][k][m] +
                             Gu[k][l][j] * Gl[i][k][m] +
                             Gu[k][i][m] * Gl[k][l][j]);
      Rt[i][j] = s;
    }

  /* conformal covariant second derivatives of phi and alpha */
  double DDphi[3][3], DDalp[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double sp = ddphi[i][j], sa = ddalp[i][j];
      for (int k = 0; k < 3; ++k) {
        sp -= Gu[k][i][j] * dphi[k];
        sa -= Gu[k][i][j] * dalp[k];
      }
      DDphi[i][j] = sp;
      DDalp[i][j] = sa;
    }
  double trDDphi = 0.0, dphi2 = 0.0, trDDalp = 0.0, dphidalp = 0.0;
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l) {
      trDDphi += gu[k][l] * DDphi[k][l];
      dphi2 += gu[k][l] * dphi[k] * dphi[l];
      trDDalp += gu[k][l] * DDalp[k][l];
      dphidalp += gu[k][l] * dphi[k] * dalp[l];
    }
  /* R^phi_ij */
  double Rphi[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      Rphi[i][j] = -2.0 * DDphi[i][j] - 2.0 * gt[i][j] * trDDphi +
                   4.0 * dphi[i] * dphi[j] - 4.0 * gt[i][j] * dphi2;

  /* raised A~ */
  double Auu[3][3], Aud[3][3]; /* A~^ij, A~^i_j */
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0, t = 0.0;
      for (int k = 0; k < 3; ++k) {
        t += gu[i][k] * At[k][j];
        for (int l = 0; l < 3; ++l) s += gu[i][k] * gu[j][l] * At[k][l];
      }
      Auu[i][j] = s;
      Aud[i][j] = t;
    }
  double AA = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) AA += At[i][j] * Auu[i][j];

  double divbeta = dbeta[0][0] + dbeta[1][1] + dbeta[2][2];
  double em4phi = exp(-4.0 * phi);

  /* gauge functions, evaluated as written */
  double f_gauge = P->lapse_f / alpha;         /* 1+log: f = 2/alpha         */
  double K0 = 0.0;
  double G_gauge = P->shift_G / (alpha * alpha); /* G = 3/(4 alpha^2)        */
  double H_gauge = exp(4.0 * phi);              /* H = exp(4 phi)            */
  double q = 1.0;
  if (P->eta_R > 0.0 && isfinite(P->eta_R)) {
    double x = g->origin[0] + p[0] * g->h[0];
    double y = g->origin[1] + p[1] * g->h[1];
    double z = g->origin[2] + p[2] * g->h[2];
    double r = sqrt(x * x + y * y + z * z);
    q = r <= P->eta_R ? 1.0 : P->eta_R / r;
  }

  double rhs[NSLOT];
  /* partial_0 phi */
  rhs[S_PHI] = -alpha * trK / 6.0 + divbeta / 6.0;
  /* partial_0 gt_ij */
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j) {
      double s = -2.0 * alpha * At[i][j];
      for (int k = 0; k < 3; ++k)
        s += gt[k][i] * dbeta[k][j] + gt[k][j] * dbeta[k][i];
      s -= 2.0 / 3.0 * gt[i][j] * divbeta;
      rhs[S_GXX + sym6(i, j)] = s;
    }
  /* partial_0 K */
  rhs[S_K] = -em4phi * (trDDalp + 2.0 * dphidalp) +
             alpha * (AA + trK * trK / 3.0);
  /* partial_0 A~_ij */
  double X[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      X[i][j] = alpha * Rt[i][j] + alpha * Rphi[i][j] - DDalp[i][j] +
                2.0 * (dphi[i] * dalp[j] + dphi[j] * dalp[i]);
  double trX = 0.0;
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l) trX += gu[k][l] * X[k][l];
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j) {
      double s = em4phi * (X[i][j] - gt[i][j] * trX / 3.0);
      s += alpha * trK * At[i][j];
      for (int k = 0; k < 3; ++k) s -= 2.0 * alpha * At[i][k] * Aud[k][j];
      for (int k = 0; k < 3; ++k)
        s += At[k][i] * dbeta[k][j] + At[k][j] * dbeta[k][i];
      s -= 2.0 / 3.0 * At[i][j] * divbeta;
      rhs[S_AXX + sym6(i, j)] = s;
    }
  /* partial_0 Gamma~^i (m = 1) */
  double T[3];
  for (int i = 0; i < 3; ++i) {
    double s = 0.0;
    for (int k = 0; k < 3; ++k)
      for (int l = 0; l < 3; ++l) s += gu[k][l] * ddbeta[i][k][l];
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) s += gu[i][j] * ddbeta[k][j][k] / 3.0;
    for (int j = 0; j < 3; ++j) s += Gd[j] * dbeta[i][j];
    s -= 2.0 / 3.0 * Gd[i] * divbeta;
    for (int j = 0; j < 3; ++j) s -= 2.0 * Auu[i][j] * dalp[j];
    double br = 0.0;
    for (int j = 0; j < 3; ++j) br += -2.0 / 3.0 * gu[i][j] * dK[j];
    for (int k = 0; k < 3; ++k)
      for (int l = 0; l < 3; ++l) br += Gu[i][k][l] * Auu[k][l];
    for (int j = 0; j < 3; ++j) br += 6.0 * Auu[i][j] * dphi[j];
    s += 2.0 * alpha * br;
    T[i] = s;
    rhs[S_GAMX + i] = s;
  }
  /* gauge */
  rhs[S_ALP] = P->lapse_static ? 0.0 : -alpha * alpha * f_gauge * (trK - K0);
  for (int i = 0; i < 3; ++i) {
    rhs[S_BETX + i] = P->shift_static ? 0.0 : alpha * alpha * G_gauge * Bv[i];
    rhs[S_BX + i] =
        P->shift_static ? 0.0 : em4phi * H_gauge * T[i] - P->eta * q * Bv[i];
  }
  rhs[S_ADOT] = 0.0;

  /* partial_t = partial_0 + beta^j partial_j (upwinded), plus dissipation */
  for (int f = 0; f < NSLOT; ++f) {
    double s = rhs[f];
    for (int ax = 0; ax < 3; ++ax)
      s += beta[ax] * dup(g, u, f, p, ax, beta[ax], ord);
    for (int ax = 0; ax < 3; ++ax) s += ko(g, u, f, p, ax, P->ko_eps, ord);
    out[f] = s;
  }
}

/* ---- argument checks shared by the entry points ------------------------ */
static int check(const oracle_grid* g, const oracle_params* P) {
  if (!g || !P) return -1;
  if (P->fd_order != 4 && P->fd_order != 8) return -1;
  int need = P->fd_order == 8 ? 5 : 3;
  if (g->ghost < need) return -1;
  for (int a = 0; a < 3; ++a)
    if (g->n[a] < 1 || !(g->h[a] > 0.0)) return -1;
  if (g->bc != 0 && g->bc != 1) return -1;
  return 0;
}

/* RHS at every interior point of u; rhs gets the interior only. */
int oracle_rhs(const oracle_grid* g, const oracle_params* P, const double* u,
               double* rhs) {
  if (check(g, P)) return -1;
  const int nx = g->n[0], ny = g->n[1], nz = g->n[2];
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        int p[3] = {i, j, k};
        double out[NSLOT];
        rhs_point(g, P, u, p, out);
        for (int f = 0; f < NSLOT; ++f) rhs[IDX(g, f, i, j, k)] = out[f];
      }
  return 0;
}

/* RHS at a list of points (interior indices, 3 per point); 25 values per
 * point written contiguously to out. */
int oracle_rhs_points(const oracle_grid* g, const oracle_params* P,
                      const double* u, int npts, const int32_t* pts,
                      double* out) {
  if (check(g, P)) return -1;
#pragma omp parallel for schedule(dynamic, 4)
  for (int t = 0; t < npts; ++t) {
    int p[3] = {pts[3 * t], pts[3 * t + 1], pts[3 * t + 2]};
    rhs_point(g, P, u, p, out + (int64_t)NSLOT * t);
  }
  return 0;
}

/* One classical RK4 step: k1..k4 are kept in separate buffers,
 *   u_{n+1} = u_n + dt/6 (k1 + 2 k2 + 2 k3 + k4).
 * Stage states reuse u_n's ghost values (static ghosts are constant in time;
 * periodic grids never read them).  u_np1 receives the whole buffer: its
 * ghosts are copied from u_n.  Buffers span slot stride * 25 elements. */
int oracle_rk4_step(const oracle_grid* g, const oracle_params* P, double dt,
                    const double* u_n, double* u_np1) {
  if (check(g, P)) return -1;
  int64_t total = g->sf * NSLOT;
  double* k[4];
  double* stage = (double*)malloc(sizeof(double) * total);
  if (!stage) return -2;
  for (int s = 0; s < 4; ++s) {
    k[s] = (double*)calloc(total, sizeof(double));
    if (!k[s]) return -2;
  }
  const double c[4] = {0.0, 0.5, 0.5, 1.0};
  const int nx = g->n[0], ny = g->n[1], nz = g->n[2];
  for (int s = 0; s < 4; ++s) {
    const double* in = u_n;
    if (s > 0) {
      memcpy(stage, u_n, sizeof(double) * total);
#pragma omp parallel for
      for (int kk = 0; kk < nz; ++kk)
        for (int j = 0; j < ny; ++j)
          for (int i = 0; i < nx; ++i)
            for (int f = 0; f < NSLOT; ++f) {
              int64_t id = IDX(g, f, i, j, kk);
              stage[id] = u_n[id] + c[s] * dt * k[s - 1][id];
            }
      in = stage;
    }
    oracle_rhs(g, P, in, k[s]);
  }
  memcpy(u_np1, u_n, sizeof(double) * total);
#pragma omp parallel for
  for (int kk = 0; kk < nz; ++kk)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i)
        for (int f = 0; f < NSLOT; ++f) {
          int64_t id = IDX(g, f, i, j, kk);
          u_np1[id] = u_n[id] + dt / 6.0 *
                                    (k[0][id] + 2.0 * k[1][id] +
                                     2.0 * k[2][id] + k[3][id]);
        }
  for (int s = 0; s < 4; ++s) free(k[s]);
  free(stage);
  return 0;
}

/* ---- constraints -----------------------------------------------------------
 * H = R - K^i_j K^j_i + K^2 and M_i = D_j K^j_i - D_i K written in the BSSN
 * variables (vacuum), assuming the algebraic conditions det gt = 1 and
 * tr A~ = 0 of the BSSN definitions:
 *   R  = e^{-4phi} g^ij (R~_ij + R^phi_ij)
 *   H  = R + 2/3 K^2 - A~_ij A~^ij
 *   M_i = d_j(g^jk A~_ik) + Gamma~^j_jk A~^k_i - Gamma~^k_ji A~^j_k
 *         + 6 A~^k_i d_k phi - 2/3 d_i K
 * and the conformal-connection constraint G^i = Gamma~^i - g^jk Gamma~^i_jk.
 */
static void constraints_point(const oracle_grid* g, const oracle_params* P,
                              const double* u, const int p[3], double* H,
                              double M[3], double Gc[3]) {
  const int ord = P->fd_order;
  double v[NSLOT];
  for (int f = 0; f < NSLOT; ++f) v[f] = U(g, u, f, p[0], p[1], p[2]);
  double gt[3][3], At[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      gt[i][j] = v[S_GXX + sym6(i, j)];
      At[i][j] = v[S_AXX + sym6(i, j)];
    }
  double det = gt[0][0] * (gt[1][1] * gt[2][2] - gt[1][2] * gt[2][1]) -
               gt[0][1] * (gt[1][0] * gt[2][2] - gt[1][2] * gt[2][0]) +
               gt[0][2] * (gt[1][0] * gt[2][1] - gt[1][1] * gt[2][0]);
  double gu[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      int r0 = (j + 1) % 3, r1 = (j + 2) % 3, c0 = (i + 1) % 3,
          c1 = (i + 2) % 3;
      gu[i][j] = (gt[r0][c0] * gt[r1][c1] - gt[r0][c1] * gt[r1][c0]) / det;
    }
  double dgt[3][3][3], dAt[3][3][3], dphi[3], dK[3], dGam[3][3];
  double ddgt[3][3][3][3], ddphi[3][3];
  for (int k = 0; k < 3; ++k) {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        dgt[i][j][k] = d1(g, u, S_GXX + sym6(i, j), p, k, ord);
        dAt[i][j][k] = d1(g, u, S_AXX + sym6(i, j), p, k, ord);
      }
    dphi[k] = d1(g, u, S_PHI, p, k, ord);
    dK[k] = d1(g, u, S_K, p, k, ord);
    for (int i = 0; i < 3; ++i) dGam[i][k] = d1(g, u, S_GAMX + i, p, k, ord);
  }
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l) {
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          ddgt[i][j][k][l] =
              k == l ? d2(g, u, S_GXX + sym6(i, j), p, k, ord)
                     : d11(g, u, S_GXX + sym6(i, j), p, k, l, ord);
      ddphi[k][l] = k == l ? d2(g, u, S_PHI, p, k, ord)
                           : d11(g, u, S_PHI, p, k, l, ord);
    }
  double Gl[3][3][3], Gu[3][3][3], dgu[3][3][3], Gd[3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k)
        Gl[i][j][k] = 0.5 * (dgt[i][j][k] + dgt[i][k][j] - dgt[j][k][i]);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) {
        double s = 0.0;
        for (int l = 0; l < 3; ++l) s += gu[i][l] * Gl[l][j][k];
        Gu[i][j][k] = s;
      }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) {
        double s = 0.0;
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) s -= gu[i][a] * gu[j][b] * dgt[a][b][k];
        dgu[i][j][k] = s;
      }
  for (int i = 0; i < 3; ++i) {
    double s = 0.0;
    for (int l = 0; l < 3; ++l) s += dgu[l][i][l];
    Gd[i] = s;
  }
  double Rt[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) s += -0.5 * gu[k][l] * ddgt[i][j][k][l];
      for (int k = 0; k < 3; ++k)
        s += 0.5 * (gt[k][i] * dGam[k][j] + gt[k][j] * dGam[k][i]);
      for (int k = 0; k < 3; ++k)
        s += -0.5 * (Gl[i][j][k] + Gl[j][i][k]) * Gd[k];
      for (int l = 0; l < 3; ++l)
        for (int m = 0; m < 3; ++m)
          for (int k = 0; k < 3; ++k)
            s += gu[l][m] * (Gu[k][l][i] * Gl[j][k][m] +
                             Gu[k][l][j] * Gl[i][k][m] +
                             Gu[k][i][m] * Gl[k][l][j]);
      Rt[i][j] = s;
    }
  double DDphi[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = ddphi[i][j];
      for (int k = 0; k < 3; ++k) s -= Gu[k][i][j] * dphi[k];
      DDphi[i][j] = s;
    }
  double trRt = 0.0, trDDphi = 0.0, dphi2 = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      trRt += gu[i][j] * Rt[i][j];
      trDDphi += gu[i][j] * DDphi[i][j];
      dphi2 += gu[i][j] * dphi[i] * dphi[j];
    }
  double Auu[3][3], Aud[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0, t = 0.0;
      for (int k = 0; k < 3; ++k) {
        t += gu[i][k] * At[k][j];
        for (int l = 0; l < 3; ++l) s += gu[i][k] * gu[j][l] * At[k][l];
      }
      Auu[i][j] = s;
      Aud[i][j] = t;
    }
  double AA = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) AA += At[i][j] * Auu[i][j];
  const double trK = v[S_K];
  double R = exp(-4.0 * v[S_PHI]) * (trRt - 8.0 * trDDphi - 8.0 * dphi2);
  *H = R + 2.0 / 3.0 * trK * trK - AA;

  for (int i = 0; i < 3; ++i) {
    /* d_j (g^jk A~_ik) by the product rule */
    double s = 0.0;
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k)
        s += dgu[j][k][j] * At[i][k] + gu[j][k] * dAt[i][k][j];
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) s += Gu[j][j][k] * Aud[k][i];
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) s -= Gu[k][j][i] * Aud[j][k];
    for (int k = 0; k < 3; ++k) s += 6.0 * Aud[k][i] * dphi[k];
    s -= 2.0 / 3.0 * dK[i];
    M[i] = s;
    double c = 0.0;
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) c += gu[j][k] * Gu[i][j][k];
    Gc[i] = v[S_GAMX + i] - c;
  }
}

/* Constraints at every interior point.  H (1 slot), M (3 slots) and Gc (3
 * slots) use the grid's layout and may be NULL.  norms[8] receives
 *   H_rms, H_max, |M|_rms, |M|_max, |G|_rms, |G|_max, N_used, N_nonfinite
 * over interior points farther than r_exc from every centre (host array of
 * 3*ncent coordinates); rms is sqrt(sum / N_used); |M| is the flat norm. */
int oracle_constraints(const oracle_grid* g, const oracle_params* P,
                       const double* u, double* H, double* M, double* Gc,
                       const double* centres, int ncent, double r_exc,
                       double* norms) {
  if (check(g, P)) return -1;
  const int nx = g->n[0], ny = g->n[1], nz = g->n[2];
  double hs = 0, hm = 0, ms = 0, mm = 0, gs = 0, gm = 0, nu = 0, nn = 0;
#pragma omp parallel for schedule(dynamic, 1) \
    reduction(+ : hs, ms, gs, nu, nn) reduction(max : hm, mm, gm)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        int p[3] = {i, j, k};
        double h, m[3], c[3];
        constraints_point(g, P, u, p, &h, m, c);
        if (H) H[IDX(g, 0, i, j, k)] = h;
        for (int a = 0; a < 3; ++a) {
          if (M) M[IDX(g, a, i, j, k)] = m[a];
          if (Gc) Gc[IDX(g, a, i, j, k)] = c[a];
        }
        int use = 1;
        double x = g->origin[0] + i * g->h[0], y = g->origin[1] + j * g->h[1],
               z = g->origin[2] + k * g->h[2];
        for (int t = 0; t < ncent; ++t) {
          double dx = x - centres[3 * t], dy = y - centres[3 * t + 1],
                 dz = z - centres[3 * t + 2];
          if (sqrt(dx * dx + dy * dy + dz * dz) <= r_exc) use = 0;
        }
        if (!use) continue;
        double mag = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
        double gmag = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        if (!isfinite(h) || !isfinite(mag) || !isfinite(gmag)) {
          nn += 1;
          continue;
        }
        nu += 1;
        hs += h * h;
        ms += mag * mag;
        gs += gmag * gmag;
        if (fabs(h) > hm) hm = fabs(h);
        if (mag > mm) mm = mag;
        if (gmag > gm) gm = gmag;
      }
  norms[0] = nu > 0 ? sqrt(hs / nu) : 0.0;
  norms[1] = hm;
  norms[2] = nu > 0 ? sqrt(ms / nu) : 0.0;
  norms[3] = mm;
  norms[4] = nu > 0 ? sqrt(gs / nu) : 0.0;
  norms[5] = gm;
  norms[6] = nu;
  norms[7] = nn;
  return 0;
}

/* Debug view of the discrete operators for one slot at one point:
 * out[0..2] first derivatives, out[3..11] second derivatives (row-major
 * 3x3), out[12..14] lopsided derivatives for the given beta signs,
 * out[15..17] Kreiss-Oliger terms per axis (with eps). */
int oracle_point_ops(const oracle_grid* g, const oracle_params* P,
                     const double* u, int f, const int32_t p_in[3],
                     const double beta[3], double* out) {
  if (check(g, P)) return -1;
  int p[3] = {p_in[0], p_in[1], p_in[2]};
  const int ord = P->fd_order;
  for (int a = 0; a < 3; ++a) out[a] = d1(g, u, f, p, a, ord);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      out[3 + 3 * a + b] = a == b ? d2(g, u, f, p, a, ord)
                                  : d11(g, u, f, p, a, b, ord);
  for (int a = 0; a < 3; ++a) out[12 + a] = dup(g, u, f, p, a, beta[a], ord);
  for (int a = 0; a < 3; ++a) out[15 + a] = ko(g, u, f, p, a, P->ko_eps, ord);
  return 0;
}

/* Number of OpenMP threads the oracle's parallel loops use. */
int oracle_num_threads(void) { return omp_get_max_threads(); }

/* Number of OpenMP threads for the following parallel loops (n >= 1). */
void oracle_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
