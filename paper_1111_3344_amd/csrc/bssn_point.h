// bssn_point.h -- the BSSN right-hand side at one grid point, templated on
// the finite-difference order (4 or 8), the arithmetic type T (double, or
// float for the mixed-precision path) and a loader L that fetches the state.
//
// Equations: vacuum BSSN, phi-variant, m = 1, with 1+log slicing and the
// Gamma-driver shift (Einstein Toolkit paper, "Spacetime Curvature
// Evolution": definitions, evolution equations, Ricci split, gauge choices
// and the attenuation q(r)).  Readings taken where the paper is silent:
//  * d_t = partial_0 + beta^j d_j with the beta^j d_j term by the lopsided
//    stencil on the side of sign(beta^j) (upwinding);
//  * Kreiss-Oliger +eps 2^-2r (-1)^(r+1) h^(2r-1) (D+D-)^r, r = 3 (order 4)
//    or 5 (order 8), on every slot and axis;
//  * d_k gt^ij = -gt^ia gt^jb d_k gt_ab (the inverse metric is never
//    differenced); the evolved Gt^i enters only as d_j Gt^k in R~_ij, every
//    other Gt^i is Gd^i = d_j gt^ji;
//  * slot A has zero source; vacuum (matter terms dropped).
//
// Numerics: every stencil works on differences from the centre value taken
// in FP64 (first derivatives on u(+k) - u(-k)), so O(1) fields carrying
// small perturbations keep their relative accuracy; in the mixed path the
// differences are rounded to FP32 only after the subtraction.  Advection and
// dissipation share one weight vector per axis, built once per point:
//   w_k = (beta * upwind_k(sign beta) + eps * ko_k) / h.
// The algebra is arranged field by field so that second derivatives are
// contracted as soon as they are formed (fewer live registers); gauge
// functions are simplified algebraically (alpha^2 * (f/alpha) = f alpha,
// alpha^2 * G/alpha^2 = shift_G, e^{-4phi} e^{4phi} = 1).
#pragma once
#include <hip/hip_runtime.h>

#include "bssn_internal.h"

namespace bssn {

// Compiler-only memory fence between field phases: keeps each slot's stencil
// loads inside its phase instead of letting the scheduler hoist hundreds of
// independent loads to the top of the kernel (which spills registers).
#define BSSN_PHASE() asm volatile("" ::: "memory")

// Materialise a value in a register here: the arithmetic producing it cannot
// sink below this point, so a phase's loads die inside the phase.
template <typename T>
__device__ __forceinline__ void keep(T& x) {
  asm volatile("" : "+v"(x));
}

// ---- stencil weights --------------------------------------------------------
template <int ORDER>
struct FD;

template <>
struct FD<4> {
  static constexpr int M = 2;  // reach of the centred operators
  static constexpr int R = 3;  // reach of upwinding and dissipation
  // centred first derivative: sum_k a(k) (u(k) - u(-k)) / h
  __host__ __device__ static constexpr double a(int k) {
    return k == 1 ? 2.0 / 3.0 : -1.0 / 12.0;
  }
  // centred second derivative: sum_k b(k) ((u(k)-u0) + (u(-k)-u0)) / h^2
  __host__ __device__ static constexpr double b(int k) {
    return k == 1 ? 4.0 / 3.0 : -1.0 / 12.0;
  }
  // lopsided first derivative for beta > 0 (offsets -1..3)
  __host__ __device__ static constexpr double up(int k) {
    return k == -1  ? -3.0 / 12.0
           : k == 0 ? -10.0 / 12.0
           : k == 1 ? 18.0 / 12.0
           : k == 2 ? -6.0 / 12.0
           : k == 3 ? 1.0 / 12.0
                    : 0.0;
  }
  // dissipation weight (sign and 2^-6 included), offsets +-1..3
  __host__ __device__ static constexpr double ko(int k) {
    return (k < 0 ? -k : k) == 1   ? 15.0 / 64.0
           : (k < 0 ? -k : k) == 2 ? -6.0 / 64.0
                                   : 1.0 / 64.0;
  }
};

template <>
struct FD<8> {
  static constexpr int M = 4;
  static constexpr int R = 5;
  __host__ __device__ static constexpr double a(int k) {
    return k == 1 ? 4.0 / 5.0
           : k == 2 ? -1.0 / 5.0
           : k == 3 ? 4.0 / 105.0
                    : -1.0 / 280.0;
  }
  __host__ __device__ static constexpr double b(int k) {
    return k == 1 ? 8.0 / 5.0
           : k == 2 ? -1.0 / 5.0
           : k == 3 ? 8.0 / 315.0
                    : -1.0 / 560.0;
  }
  // offsets -3..5
  __host__ __device__ static constexpr double up(int k) {
    return k == -3  ? -1.0 / 168.0
           : k == -2 ? 1.0 / 14.0
           : k == -1 ? -1.0 / 2.0
           : k == 0  ? -9.0 / 20.0
           : k == 1  ? 5.0 / 4.0
           : k == 2  ? -1.0 / 2.0
           : k == 3  ? 1.0 / 6.0
           : k == 4  ? -1.0 / 28.0
           : k == 5  ? 1.0 / 280.0
                     : 0.0;
  }
  __host__ __device__ static constexpr double ko(int k) {
    return (k < 0 ? -k : k) == 1   ? 210.0 / 1024.0
           : (k < 0 ? -k : k) == 2 ? -120.0 / 1024.0
           : (k < 0 ? -k : k) == 3 ? 45.0 / 1024.0
           : (k < 0 ? -k : k) == 4 ? -10.0 / 1024.0
                                   : 1.0 / 1024.0;
  }
};

// Order in which point_rhs visits the slots (one phase per slot).  Slots
// that only need advection and dissipation (A~, B, A) alternate with the
// heavy ones, so that the time between a prefetch and its use stays even.
constexpr int kPhaseSlot[NSLOT] = {GXX,  AXX,  GXY, AXY, GXZ,  AXZ,  GYY,
                                   AYY,  GYZ,  AYZ, GZZ, AZZ,  GAMX, BX,
                                   GAMY, BY,   GAMZ, BZ, PHI,  ADOT, TRK,
                                   ALP,  BETX, BETY, BETZ};
// inverse of kPhaseSlot (a formula, so it folds after unrolling)
__host__ __device__ constexpr int phase_of(int slot) {
  return slot >= GXX && slot <= GZZ   ? 2 * (slot - GXX)
         : slot >= AXX && slot <= AZZ ? 2 * (slot - AXX) + 1
         : slot >= GAMX && slot <= GAMZ ? 12 + 2 * (slot - GAMX)
         : slot >= BX && slot <= BZ     ? 13 + 2 * (slot - BX)
         : slot == PHI                  ? 18
         : slot == ADOT                 ? 19
         : slot == TRK                  ? 20
         : slot == ALP                  ? 21
                                        : 22 + (slot - BETX);
}

// symmetric pair -> 0..5 (xx xy xz yy yz zz)
__host__ __device__ constexpr int S_(int i, int j) {  // i <= j
  return i == 0 ? j : (i == 1 ? 2 + j : 5);
}
__host__ __device__ constexpr int S(int i, int j) {
  return i <= j ? S_(i, j) : S_(j, i);
}

// ---- stencil helpers ----------------------------------------------------------
// weights index: k = -R..-1 -> 0..R-1, k = 1..R -> R..2R-1
template <int R>
__host__ __device__ constexpr int WI(int k) {
  return k < 0 ? k + R : k + R - 1;
}

// Star of one slot: first derivatives d1 (optional), pure second derivatives
// d2 (optional) and the advection + dissipation sum, on the 2R+1 points of
// each axis.
template <int ORDER, typename T, bool D1, bool D2, class L>
__device__ __forceinline__ T star(const L& ld, int s,
                                  const T (&cw)[3][2 * FD<ORDER>::R],
                                  const T (&ih)[3], const T (&ih2)[3], T* d1,
                                  T* d2) {
  using F = FD<ORDER>;
  constexpr int R = F::R, M = F::M;
  const double c0 = ld.c(s);
  T adv = T(0);
  // raw taps of two axes (index WI<R>(k)): the taps of axis a + 1 are read
  // before the arithmetic of axis a, so that their LDS latency hides behind
  // it
  double u[2][2 * R];
#pragma unroll
  for (int k = -R; k <= R; ++k)
    if (k != 0) u[0][WI<R>(k)] = ld.ax(s, 0, k);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a < 2) {
#pragma unroll
      for (int k = -R; k <= R; ++k)
        if (k != 0) u[(a + 1) & 1][WI<R>(k)] = ld.ax(s, a + 1, k);
    }
    double d[2 * R + 1];
#pragma unroll
    for (int k = -R; k <= R; ++k)
      if (k != 0) d[R + k] = u[a & 1][WI<R>(k)] - c0;
    if constexpr (D1) {
      T s1 = T(0);
#pragma unroll
      for (int k = 1; k <= M; ++k)
        s1 += T(F::a(k)) * T(d[R + k] - d[R - k]);
      d1[a] = s1 * ih[a];
      keep(d1[a]);
    }
    if constexpr (D2) {
      T s2 = T(0);
#pragma unroll
      for (int k = 1; k <= M; ++k)
        s2 += T(F::b(k)) * T(d[R + k] + d[R - k]);
      d2[a] = s2 * ih2[a];
      keep(d2[a]);
    }
    // two independent chains (taps below and above the point), so that
    // the FMA latency of one hides behind the other
    T lo = T(0), hi = T(0);
#pragma unroll
    for (int k = 1; k <= R; ++k) {
      lo += cw[a][WI<R>(-k)] * T(d[R - k]);
      hi += cw[a][WI<R>(k)] * T(d[R + k]);
    }
    adv += lo + hi;
    keep(adv);
  }
  return adv;
}

// Mixed second derivative d_a d_b (a != b): tensor product of the centred
// first-derivative stencils, nested on pairwise differences.
template <int ORDER, typename T, class L>
__device__ __forceinline__ T mixed(const L& ld, int s, int a, int b, T ihab) {
  using F = FD<ORDER>;
  constexpr int M = F::M;
  T acc = T(0);
#pragma unroll
  for (int i = 1; i <= M; ++i) {
    T p = T(0), m = T(0);
#pragma unroll
    for (int j = 1; j <= M; ++j) {
      p += T(F::a(j)) * T(ld.pl(s, a, i, b, j) - ld.pl(s, a, i, b, -j));
      m += T(F::a(j)) * T(ld.pl(s, a, -i, b, j) - ld.pl(s, a, -i, b, -j));
    }
    acc += T(F::a(i)) * (p - m);
  }
  T v = acc * ihab;
  keep(v);
  return v;
}

// Loaders that form the three mixed derivatives of a slot together (sharing
// inner sums across the tile) declare kSharedMixed = true and mixed3().
template <class L, class = void>
struct SharedMixed {
  static constexpr bool value = false;
};
template <class L>
struct SharedMixed<L, decltype(void(L::kSharedMixed))> {
  static constexpr bool value = L::kSharedMixed;
};

// d_x d_y, d_x d_z, d_y d_z of slot s at the point.
template <int ORDER, typename T, class L>
__device__ __forceinline__ void mixed_all(const L& ld, int s, T ihxy, T ihxz,
                                          T ihyz, T& dxy, T& dxz, T& dyz) {
  if constexpr (SharedMixed<L>::value) {
    ld.template mixed3<ORDER, T>(ihxy, ihxz, ihyz, dxy, dxz, dyz);
  } else {
    dxy = mixed<ORDER, T>(ld, s, 0, 1, ihxy);
    dxz = mixed<ORDER, T>(ld, s, 0, 2, ihxz);
    dyz = mixed<ORDER, T>(ld, s, 1, 2, ihyz);
  }
}

template <typename T>
__device__ __forceinline__ T t_exp(T x);
template <>
__device__ __forceinline__ double t_exp<double>(double x) {
  return exp(x);
}
template <>
__device__ __forceinline__ float t_exp<float>(float x) {
  return expf(x);
}

// ---- the right-hand side at one point --------------------------------------------
// ih: 1/h per axis; (xc, yc, zc): coordinates of the point (for q(r)).
// Loader interface: g(s) centre value of slot s (any slot, any time);
// enter(s) starts the phase of slot s (slots are entered in the order of
// kPhaseSlot); c(s), ax(s, a, k), pl(s, a, i, b, j) read slot s inside its
// phase (centre, offset k along axis a, offsets i along a and j along b).
// Sp: inverse spacings ih[3], ih2[3], ihm[3] (xy, xz, yz), uniform.
template <int ORDER, typename T, class L, class Sp>
__device__ __forceinline__ void point_rhs(const L& ld, const Sp& sp,
                                          double xc, double yc, double zc,
                                          const Gauge& G, T (&r)[NSLOT]) {
  using F = FD<ORDER>;
  constexpr int R = F::R;
  T ih[3], ih2[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    ih[a] = T(sp.ih[a]);
    ih2[a] = T(sp.ih2[a]);
  }
  const T ihxy = T(sp.ihm[0]), ihxz = T(sp.ihm[1]), ihyz = T(sp.ihm[2]);

  // centre values needed from the start: gt_ij, beta^i, alpha
  T gt[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) gt[m] = T(ld.g(GXX + m));
  const T alpha = T(ld.g(ALP));

  // inverse conformal metric (adjugate / determinant)
  const T c00 = gt[3] * gt[5] - gt[4] * gt[4];
  const T c01 = gt[2] * gt[4] - gt[1] * gt[5];
  const T c02 = gt[1] * gt[4] - gt[2] * gt[3];
  const T idet = T(1) / (gt[0] * c00 + gt[1] * c01 + gt[2] * c02);
  T gu[6];
  gu[0] = c00 * idet;
  gu[1] = c01 * idet;
  gu[2] = c02 * idet;
  gu[3] = (gt[0] * gt[5] - gt[2] * gt[2]) * idet;
  gu[4] = (gt[1] * gt[2] - gt[0] * gt[4]) * idet;
  gu[5] = (gt[0] * gt[3] - gt[1] * gt[1]) * idet;

  // advection + dissipation weights per axis
  T cw[3][2 * R];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double bb = ld.g(BETX + a);
    const bool pos = bb > 0.0;
#pragma unroll
    for (int k = -R; k <= R; ++k) {
      if (k == 0) continue;
      const double W = pos ? F::up(k) : -F::up(-k);
      cw[a][WI<R>(k)] = T((bb * W + G.ko_eps * F::ko(k)) * sp.ih[a]);
    }
  }

  // ---- gt_ij (first derivatives; trace of the second derivatives into
  //      R~), alternating with A~_ij (advection only; centre value kept) --
  T dgt[6][3];
  T Rt[6];
  T At[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    T d2[3];
    ld.enter(GXX + m);
    r[GXX + m] =
        star<ORDER, T, true, true>(ld, GXX + m, cw, ih, ih2, dgt[m], d2);
    BSSN_PHASE();
    T dxy, dxz, dyz;
    mixed_all<ORDER, T>(ld, GXX + m, ihxy, ihxz, ihyz, dxy, dxz, dyz);
    Rt[m] = T(-0.5) * (gu[0] * d2[0] + gu[3] * d2[1] + gu[5] * d2[2] +
                       T(2) * (gu[1] * dxy + gu[2] * dxz + gu[4] * dyz));
    keep(Rt[m]);
    ld.enter(AXX + m);
    At[m] = T(ld.c(AXX + m));
    r[AXX + m] = star<ORDER, T, false, false>(ld, AXX + m, cw, ih, ih2,
                                              nullptr, nullptr);
  }

  // Christoffel symbols: Gl[i][S(j,k)] = Gamma~_ijk, Gu[i][S(j,k)] =
  // Gamma~^i_jk
  T Gl[3][6], Gu[3][6];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = j; k < 3; ++k)
        Gl[i][S(j, k)] = T(0.5) * (dgt[S(i, j)][k] + dgt[S(i, k)][j] -
                                   dgt[S(j, k)][i]);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int m = 0; m < 6; ++m)
      Gu[i][m] = gu[S(i, 0)] * Gl[0][m] + gu[S(i, 1)] * Gl[1][m] +
                 gu[S(i, 2)] * Gl[2][m];
  // Gd^i = d_l gt^li = -gt^ib Q_b, Q_b = gt^la d_l gt_ab
  T Gd[3];
  {
    T Q[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      T s = T(0);
#pragma unroll
      for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int a = 0; a < 3; ++a) s += gu[S(l, a)] * dgt[S(a, b)][l];
      Q[b] = s;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
      Gd[i] = -(gu[S(i, 0)] * Q[0] + gu[S(i, 1)] * Q[1] + gu[S(i, 2)] * Q[2]);
  }
  // quadratic Ricci terms, one k at a time:
  //   gt^lm (G^k_li G_jkm + G^k_lj G_ikm + G^k_im G_klj)
  //   = sum_k sum_m [ H3_k[m][i] Gl_jkm + H3_k[m][j] Gl_ikm
  //                  + G^k_im H2_k[m][j] ]
  // with H3_k[m][i] = gt^ml G^k_li and H2_k[m][j] = gt^ml G_klj, and
  //   - (Gl_ijk + Gl_jik) Gd^k / 2
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T H3[3][3], H2[3][3];
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        H3[m][i] = gu[S(m, 0)] * Gu[k][S(0, i)] + gu[S(m, 1)] * Gu[k][S(1, i)] +
                   gu[S(m, 2)] * Gu[k][S(2, i)];
        H2[m][i] = gu[S(m, 0)] * Gl[k][S(0, i)] + gu[S(m, 1)] * Gl[k][S(1, i)] +
                   gu[S(m, 2)] * Gl[k][S(2, i)];
      }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) {
        T s = -T(0.5) * (Gl[i][S(j, k)] + Gl[j][S(i, k)]) * Gd[k];
#pragma unroll
        for (int m = 0; m < 3; ++m)
          s += H3[m][i] * Gl[j][S(k, m)] + H3[m][j] * Gl[i][S(k, m)] +
               Gu[k][S(i, m)] * H2[m][j];
        Rt[S(i, j)] += s;
        keep(Rt[S(i, j)]);
      }
  }

  // ---- Gt^k (d_j Gt^k into R~_ij), alternating with B^k --------------------
  T Bv[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T dG[3];
    ld.enter(GAMX + k);
    r[GAMX + k] =
        star<ORDER, T, true, false>(ld, GAMX + k, cw, ih, ih2, dG, nullptr);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j)
        Rt[S(i, j)] += T(0.5) * (gt[S(k, i)] * dG[j] + gt[S(k, j)] * dG[i]);
    ld.enter(BX + k);
    Bv[k] = T(ld.c(BX + k));
    r[BX + k] = star<ORDER, T, false, false>(ld, BX + k, cw, ih, ih2, nullptr,
                                             nullptr);
  }

  // ---- phi: R^phi_ij into R~_ij ------------------------------------------------
  T dphi[3];
  ld.enter(PHI);
  const T phi = T(ld.c(PHI));
  {
    T d2[3];
    r[PHI] = star<ORDER, T, true, true>(ld, PHI, cw, ih, ih2, dphi, d2);
    T dd[6];
    dd[0] = d2[0];
    dd[3] = d2[1];
    dd[5] = d2[2];
    BSSN_PHASE();
    mixed_all<ORDER, T>(ld, PHI, ihxy, ihxz, ihyz, dd[1], dd[2], dd[4]);
    T DD[6];
#pragma unroll
    for (int m = 0; m < 6; ++m)
      DD[m] = dd[m] - (Gu[0][m] * dphi[0] + Gu[1][m] * dphi[1] +
                       Gu[2][m] * dphi[2]);
    const T trDD = gu[0] * DD[0] + gu[3] * DD[3] + gu[5] * DD[5] +
                   T(2) * (gu[1] * DD[1] + gu[2] * DD[2] + gu[4] * DD[4]);
    const T dphi2 =
        gu[0] * dphi[0] * dphi[0] + gu[3] * dphi[1] * dphi[1] +
        gu[5] * dphi[2] * dphi[2] +
        T(2) * (gu[1] * dphi[0] * dphi[1] + gu[2] * dphi[0] * dphi[2] +
                gu[4] * dphi[1] * dphi[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) {
        const int m = S(i, j);
        Rt[m] += T(-2) * DD[m] - T(2) * gt[m] * trDD +
                 T(4) * dphi[i] * dphi[j] - T(4) * gt[m] * dphi2;
      }
  }

  // ---- A (advection only) ------------------------------------------------------
  ld.enter(ADOT);
  r[ADOT] = star<ORDER, T, false, false>(ld, ADOT, cw, ih, ih2, nullptr,
                                         nullptr);

  // ---- K: the -4/3 alpha gt^ij d_j K part of Gt's source ----------------------
  T Tg[3];
  ld.enter(TRK);
  const T trK = T(ld.c(TRK));
  {
    T dK[3];
    r[TRK] = star<ORDER, T, true, false>(ld, TRK, cw, ih, ih2, dK, nullptr);
#pragma unroll
    for (int i = 0; i < 3; ++i)
      Tg[i] = T(-4.0 / 3.0) * alpha *
              (gu[S(i, 0)] * dK[0] + gu[S(i, 1)] * dK[1] + gu[S(i, 2)] * dK[2]);
  }

  // ---- alpha: X_ij, the A~ and K sources, the rest of Gt's source ---------
  ld.enter(ALP);
  {
    T dalp[3], d2[3];
    r[ALP] = star<ORDER, T, true, true>(ld, ALP, cw, ih, ih2, dalp, d2);
    T dd[6];
    dd[0] = d2[0];
    dd[3] = d2[1];
    dd[5] = d2[2];
    BSSN_PHASE();
    mixed_all<ORDER, T>(ld, ALP, ihxy, ihxz, ihyz, dd[1], dd[2], dd[4]);
    const T em4phi = t_exp<T>(T(-4) * phi);
    // A~^i_j, A~^ij and A~_ij A~^ij
    T Aud[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        Aud[i][j] = gu[S(i, 0)] * At[S(0, j)] + gu[S(i, 1)] * At[S(1, j)] +
                    gu[S(i, 2)] * At[S(2, j)];
    T Auu[6];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j)
        Auu[S(i, j)] = Aud[i][0] * gu[S(0, j)] + Aud[i][1] * gu[S(1, j)] +
                       Aud[i][2] * gu[S(2, j)];
    const T AA = At[0] * Auu[0] + At[3] * Auu[3] + At[5] * Auu[5] +
                 T(2) * (At[1] * Auu[1] + At[2] * Auu[2] + At[4] * Auu[4]);
    T DD[6], X[6];
#pragma unroll
    for (int m = 0; m < 6; ++m)
      DD[m] = dd[m] - (Gu[0][m] * dalp[0] + Gu[1][m] * dalp[1] +
                       Gu[2][m] * dalp[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) {
        const int m = S(i, j);
        X[m] = alpha * Rt[m] - DD[m] +
               T(2) * (dphi[i] * dalp[j] + dphi[j] * dalp[i]);
      }
    const T trX = gu[0] * X[0] + gu[3] * X[3] + gu[5] * X[5] +
                  T(2) * (gu[1] * X[1] + gu[2] * X[2] + gu[4] * X[4]);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) {
        const int m = S(i, j);
        T s = em4phi * (X[m] - gt[m] * trX * T(1.0 / 3.0)) +
              alpha * trK * At[m];
        s -= T(2) * alpha *
             (At[S(i, 0)] * Aud[0][j] + At[S(i, 1)] * Aud[1][j] +
              At[S(i, 2)] * Aud[2][j]);
        r[AXX + m] += s;
      }
    const T trDD = gu[0] * DD[0] + gu[3] * DD[3] + gu[5] * DD[5] +
                   T(2) * (gu[1] * DD[1] + gu[2] * DD[2] + gu[4] * DD[4]);
    const T dpda =
        gu[0] * dphi[0] * dalp[0] + gu[3] * dphi[1] * dalp[1] +
        gu[5] * dphi[2] * dalp[2] +
        gu[1] * (dphi[0] * dalp[1] + dphi[1] * dalp[0]) +
        gu[2] * (dphi[0] * dalp[2] + dphi[2] * dalp[0]) +
        gu[4] * (dphi[1] * dalp[2] + dphi[2] * dalp[1]);
    r[TRK] += -em4phi * (trDD + T(2) * dpda) +
              alpha * (AA + trK * trK * T(1.0 / 3.0));
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const T GA = Gu[i][0] * Auu[0] + Gu[i][3] * Auu[3] + Gu[i][5] * Auu[5] +
                   T(2) * (Gu[i][1] * Auu[1] + Gu[i][2] * Auu[2] +
                           Gu[i][4] * Auu[4]);
      const T Ad = Auu[S(i, 0)] * dalp[0] + Auu[S(i, 1)] * dalp[1] +
                   Auu[S(i, 2)] * dalp[2];
      const T Ap = Auu[S(i, 0)] * dphi[0] + Auu[S(i, 1)] * dphi[1] +
                   Auu[S(i, 2)] * dphi[2];
      Tg[i] += T(-2) * Ad + T(2) * alpha * (GA + T(6) * Ap);
    }
  }

  // ---- beta^k: shift terms of gt, A~, Gt ------------------------------------
  T rg[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) rg[m] = T(0);
  T V[3] = {T(0), T(0), T(0)};
  T divb = T(0);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T db[3], d2[3];
    ld.enter(BETX + k);
    r[BETX + k] =
        star<ORDER, T, true, true>(ld, BETX + k, cw, ih, ih2, db, d2);
    T dd[6];
    dd[0] = d2[0];
    dd[3] = d2[1];
    dd[5] = d2[2];
    BSSN_PHASE();
    mixed_all<ORDER, T>(ld, BETX + k, ihxy, ihxz, ihyz, dd[1], dd[2], dd[4]);
    Tg[k] += gu[0] * dd[0] + gu[3] * dd[3] + gu[5] * dd[5] +
             T(2) * (gu[1] * dd[1] + gu[2] * dd[2] + gu[4] * dd[4]);
    Tg[k] += Gd[0] * db[0] + Gd[1] * db[1] + Gd[2] * db[2];
#pragma unroll
    for (int j = 0; j < 3; ++j) V[j] += dd[S(j, k)];
    divb += db[k];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) {
        rg[S(i, j)] += gt[S(k, i)] * db[j] + gt[S(k, j)] * db[i];
        r[AXX + S(i, j)] += At[S(k, i)] * db[j] + At[S(k, j)] * db[i];
      }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
    Tg[i] += T(1.0 / 3.0) * (gu[S(i, 0)] * V[0] + gu[S(i, 1)] * V[1] +
                             gu[S(i, 2)] * V[2]) -
             T(2.0 / 3.0) * Gd[i] * divb;
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    r[GXX + m] += rg[m] - T(2) * alpha * At[m] - T(2.0 / 3.0) * gt[m] * divb;
    r[AXX + m] -= T(2.0 / 3.0) * At[m] * divb;
  }
  r[PHI] += (divb - alpha * trK) * T(1.0 / 6.0);

  // ---- gauge ---------------------------------------------------------------------
#pragma unroll
  for (int i = 0; i < 3; ++i) r[GAMX + i] += Tg[i];
  if (!G.lapse_static) r[ALP] -= T(G.lapse_f) * alpha * trK;
  if (!G.shift_static) {
    T q = T(1);
    if (G.eta_R > 0.0) {
      const double rad = sqrt(xc * xc + yc * yc + zc * zc);
      q = T(rad <= G.eta_R ? 1.0 : G.eta_R / rad);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      r[BETX + i] += T(G.shift_G) * Bv[i];
      r[BX + i] += Tg[i] - T(G.eta) * q * Bv[i];
    }
  }
}

}  // namespace bssn
