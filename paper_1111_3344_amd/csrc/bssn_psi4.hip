// bssn_psi4.hip -- the Weyl scalar Psi_4 on the grid (Einstein Toolkit
// paper, section "Analysis", gravitational waves: the WeylScal4 module).
//
// Psi_4 = C_abcd n^a mb^b n^c mb^d on the fiducial tetrad
//   l = (u + rhat)/sqrt2, n = (u - rhat)/sqrt2, m = (thetahat + i phihat)/sqrt2,
// u the unit normal of the slice, the spatial triad started from
// phi~ = (-y, x, 0), r~ = (x, y, z), theta~^i = sqrt(det g) g^ik eps_klm
// phi~^l r~^m (coordinates relative to a given centre) and made orthonormal
// with the 3-metric by Gram-Schmidt, phi first, then r, then theta.  In
// vacuum the Weyl tensor is the Riemann tensor, whose projections follow
// from the 3+1 data by the Gauss, Codazzi and Ricci equations with
// K_ij = -(1/2) L_u g_ij (the sign of d_t g_ij = -2 alpha K_ij + ...):
//   R_ijkl (spatial)  = 3R_ijkl + K_ik K_jl - K_il K_jk,
//   R_ujkl            = D_k K_jl - D_l K_jk,
//   R_ujul            = g^ik R_ijkl (spatial, the line above),
// the last because the 4-Ricci tensor vanishes.  The tetrad's m has no
// component along u, so with n = (u - rhat)/sqrt2
//   Psi_4 = R_ijkl n^i mb^j n^k mb^l + sqrt2 R_ujkl mb^j n^k mb^l
//           + (1/2) R_ujul mb^j mb^l.
//
// How it is evaluated here (differently arranged from the plain contraction
// of the paper's formula, equal to it up to rounding):
//  * the ADM metric g_ij = e^{4 phi} gt_ij and curvature
//    K_ij = e^{4 phi} (At_ij + gt_ij K/3) come from the BSSN state by
//    inverting the paper's definitions, at every point of a tile's box;
//  * their derivatives are the evolution's centred stencils on g (first,
//    pure second, and mixed = product of first-derivative stencils) and on
//    K (first), formed from the box in LDS;
//  * in 3-D the Riemann tensor has the six components R_PQ over the index
//    pairs P, Q in {xy, xz, yz}, so R_ijkl n^i mb^j n^k mb^l is
//    sum_PQ R_PQ B^P B^Q with the bivector B^ij = n^i mb^j - n^j mb^i.
//
// One workgroup of 256 threads per 16 x 4 x 4 tile (one point per thread,
// wave w = plane w of the tile); tiles are numbered x fastest and dealt to
// the XCDs in contiguous eighths, so neighbouring tiles share an L2.  The
// box (tile + M = order/2 on every side) holds e^{4 phi} and K/3 for the
// whole pass (each thread re-reads only its own entries; at order 8 they
// are kept in registers instead) and, per symmetric
// component, g_ij and K_ij, converted on the way from memory into LDS.
// Algorithmic bytes: 14 slots in (phi, gt_ij, K, At_ij), 2 out (re, im):
// 128 B per interior point.  Roofline: HBM.
#include <hip/hip_runtime.h>

#include "bssn_internal.h"
#include "bssn_kernels.h"

namespace bssn {
namespace {

constexpr int TX = 16, TY = 4, TZ = 4;

template <int ORDER>
struct Box {
  static constexpr int M = ORDER / 2;
  static constexpr int X = TX + 2 * M, Y = TY + 2 * M, Z = TZ + 2 * M;
  static constexpr int N = X * Y * Z;
};

// centred stencil weights: first derivative on u(+k) - u(-k), second on
// u(+k) + u(-k) - 2 u(0), k = 1..order/2
template <int ORDER>
__device__ __forceinline__ constexpr double wa(int k) {
  return ORDER == 4 ? (k == 1 ? 2.0 / 3.0 : -1.0 / 12.0)
                    : (k == 1   ? 4.0 / 5.0
                       : k == 2 ? -1.0 / 5.0
                       : k == 3 ? 4.0 / 105.0
                                : -1.0 / 280.0);
}
template <int ORDER>
__device__ __forceinline__ constexpr double wb(int k) {
  return ORDER == 4 ? (k == 1 ? 4.0 / 3.0 : -1.0 / 12.0)
                    : (k == 1   ? 8.0 / 5.0
                       : k == 2 ? -1.0 / 5.0
                       : k == 3 ? 8.0 / 315.0
                                : -1.0 / 560.0);
}

// symmetric pair -> 0..5 (xx xy xz yy yz zz)
__device__ __forceinline__ constexpr int sy6(int i, int j) {
  const int a = i < j ? i : j, b = i < j ? j : i;
  return a == 0 ? b : (a == 1 ? 2 + b : 5);
}
// antisymmetric pair i < j -> 0..2 (xy xz yz)
__device__ __forceinline__ constexpr int ap(int i, int j) {
  return i == 0 ? j - 1 : 2;
}

struct C2 {  // complex double
  double re, im;
};
__device__ __forceinline__ C2 cmul(C2 a, C2 b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ C2 cscale(C2 a, double s) {
  return {a.re * s, a.im * s};
}
__device__ __forceinline__ C2 cadd(C2 a, C2 b) {
  return {a.re + b.re, a.im + b.im};
}

// R_ijkl for any indices from the pair components R[P][Q]
__device__ __forceinline__ double rpair(const double (&R)[3][3], int i, int j,
                                        int k, int l) {
  if (i == j || k == l) return 0.0;
  const double s = (i < j ? 1.0 : -1.0) * (k < l ? 1.0 : -1.0);
  const int P = i < j ? ap(i, j) : ap(j, i);
  const int Q = k < l ? ap(k, l) : ap(l, k);
  return s * R[P][Q];
}

// g_ij a^i b^j
__device__ __forceinline__ double gdot(const double (&g)[6],
                                       const double (&a)[3],
                                       const double (&b)[3]) {
  return g[0] * a[0] * b[0] + g[3] * a[1] * b[1] + g[5] * a[2] * b[2] +
         g[1] * (a[0] * b[1] + a[1] * b[0]) +
         g[2] * (a[0] * b[2] + a[2] * b[0]) +
         g[4] * (a[1] * b[2] + a[2] * b[1]);
}

// e^{4 phi} and K/3 at this thread's box points (each thread reads only the
// entries it wrote, so no barrier guards them): in registers (REG, order 8,
// which frees LDS for a second workgroup per CU) or in LDS (order 4, whose
// registers are needed for two waves per SIMD).
template <bool REG, int NP>
struct BoxScalars;
template <int NP>
struct BoxScalars<true, NP> {
  double e[NP], k[NP];
  __device__ __forceinline__ void set(int q, int, double ev, double kv) {
    e[q] = ev;
    k[q] = kv;
  }
  __device__ __forceinline__ double e4(int q, int) const { return e[q]; }
  __device__ __forceinline__ double k3(int q, int) const { return k[q]; }
};
template <int NP>
struct BoxScalars<false, NP> {
  double* e;
  double* k;
  __device__ __forceinline__ void set(int, int p, double ev, double kv) {
    e[p] = ev;
    k[p] = kv;
  }
  __device__ __forceinline__ double e4(int, int p) const { return e[p]; }
  __device__ __forceinline__ double k3(int, int p) const { return k[p]; }
};

// Everything a point keeps from the six component passes.
struct Acc {
  double gm[6], K[6], dg[3][6], dK[3][6];
  double R[3][3];  // second-derivative part of the Riemann pair components
};

constexpr int PI[3] = {0, 0, 1}, PJ[3] = {1, 2, 2};  // pair P = (PI, PJ)

// One symmetric component C of g_ij and K_ij: convert the box from memory
// into LDS, then form this point's value, first derivatives and (into the
// Riemann pair components) second derivatives.
template <int ORDER, int C, int NP, class BS>
__device__ __forceinline__ void component(Acc& a, const double* u, int64_t sf,
                                          const int32_t (&sidx)[NP], int t,
                                          int c0, const double (&ih)[3],
                                          const BS& bs, double* gs,
                                          double* ks) {
  using B = Box<ORDER>;
  constexpr int M = B::M;
  constexpr int st[3] = {1, B::X, B::X * B::Y};
  // g_ij and K_ij of component c over the box
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const int p = t + 256 * q;
    if (p < B::N) {
      double gv = 0.0, kv = 0.0;
      if (sidx[q] >= 0) {
        const double gt = u[(GXX + C) * sf + sidx[q]];
        const double at = u[(AXX + C) * sf + sidx[q]];
        gv = bs.e4(q, p) * gt;
        kv = bs.e4(q, p) * (at + gt * bs.k3(q, p));
      }
      gs[p] = gv;
      ks[p] = kv;
    }
  }
  __syncthreads();
  const double g0 = gs[c0];
  a.gm[C] = g0;
  a.K[C] = ks[c0];
  double dd[6];
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    double s1 = 0.0, s2 = 0.0, sk = 0.0;
#pragma unroll
    for (int k = 1; k <= M; ++k) {
      const double gp = gs[c0 + k * st[x]], gmn = gs[c0 - k * st[x]];
      s1 += wa<ORDER>(k) * (gp - gmn);
      s2 += wb<ORDER>(k) * ((gp - g0) + (gmn - g0));
      sk += wa<ORDER>(k) * (ks[c0 + k * st[x]] - ks[c0 - k * st[x]]);
    }
    asm volatile("" : "+v"(s1), "+v"(s2), "+v"(sk)::"memory");
    a.dg[x][C] = s1 * ih[x];
    dd[sy6(x, x)] = s2 * ih[x] * ih[x];
    a.dK[x][C] = sk * ih[x];
  }
#pragma unroll
  for (int y = 0; y < 3; ++y)
#pragma unroll
    for (int b = y + 1; b < 3; ++b) {
      double s = 0.0;
#pragma unroll
      for (int i = 1; i <= M; ++i) {
        double in = 0.0;
#pragma unroll
        for (int j = 1; j <= M; ++j) {
          const int pp = c0 + i * st[y] + j * st[b];
          const int pm = c0 + i * st[y] - j * st[b];
          const int mp = c0 - i * st[y] + j * st[b];
          const int mm = c0 - i * st[y] - j * st[b];
          in += wa<ORDER>(j) * ((gs[pp] - gs[pm]) - (gs[mp] - gs[mm]));
        }
        s += wa<ORDER>(i) * in;
        // compiler-only fence: keeps each row's LDS reads inside its row
        // instead of hoisting all of them (which spills registers)
        asm volatile("" : "+v"(s)::"memory");
      }
      dd[sy6(y, b)] = s * ih[y] * ih[b];
    }
#pragma unroll
  for (int P = 0; P < 3; ++P)
#pragma unroll
    for (int Q = P; Q < 3; ++Q) {
      const int i = PI[P], j = PJ[P], k = PI[Q], l = PJ[Q];
      if (sy6(i, l) == C) a.R[P][Q] += 0.5 * dd[sy6(j, k)];
      if (sy6(j, k) == C) a.R[P][Q] += 0.5 * dd[sy6(i, l)];
      if (sy6(j, l) == C) a.R[P][Q] -= 0.5 * dd[sy6(i, k)];
      if (sy6(i, k) == C) a.R[P][Q] -= 0.5 * dd[sy6(j, l)];
    }
  __syncthreads();
}

template <int ORDER>
__global__ void __launch_bounds__(256) k_psi4(const Psi4Args A) {
  using B = Box<ORDER>;
  constexpr int M = B::M;
  constexpr bool kReg = ORDER == 8;
  __shared__ double gs[B::N], ks[B::N];
  __shared__ double lds_scalars[kReg ? 2 : 2 * B::N];

  // tile of this workgroup: the XCD (block id mod 8) takes a contiguous
  // eighth of the x-fastest tile numbering
  const int ntx = (A.n[0] + TX - 1) / TX, nty = (A.n[1] + TY - 1) / TY,
            ntz = (A.n[2] + TZ - 1) / TZ;
  const int64_t ntile = int64_t(ntx) * nty * ntz;
  const int64_t per = (ntile + 7) / 8;
  const int64_t tile = int64_t(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (tile >= ntile) return;
  const int tx0 = int(tile % ntx) * TX;
  const int ty0 = int((tile / ntx) % nty) * TY;
  const int tz0 = int(tile / (int64_t(ntx) * nty)) * TZ;

  const int g = A.ghost;
  const int ex = A.n[0] + 2 * g, ey = A.n[1] + 2 * g, ez = A.n[2] + 2 * g;
  // storage coordinates of box point 0
  const int bx0 = g + tx0 - M, by0 = g + ty0 - M, bz0 = g + tz0 - M;
  const int t = threadIdx.x;

  // box points of this thread: p = t, t + 256, ...; storage index (a slot
  // is below 2 GiB, so it fits 32 bits) or -1 outside the storage grid
  constexpr int NP = (B::N + 255) / 256;
  int32_t sidx[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const int p = t + 256 * q;
    sidx[q] = -1;
    if (p < B::N) {
      const int i = p % B::X, j = (p / B::X) % B::Y, k = p / (B::X * B::Y);
      const int sx = bx0 + i, syy = by0 + j, sz = bz0 + k;
      if (sx < ex && syy < ey && sz < ez)
        sidx[q] = int32_t(int64_t(sz) * A.sz + int64_t(syy) * A.sy + sx);
    }
  }
  const double* u = A.u;
  const int64_t sf = A.sf;
  BoxScalars<kReg, NP> bs;
  if constexpr (!kReg) {
    bs.e = lds_scalars;
    bs.k = lds_scalars + B::N;
  }
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const int p = t + 256 * q;
    if (p < B::N) {
      double e = 0.0, k3 = 0.0;
      if (sidx[q] >= 0) {
        e = exp(4.0 * u[PHI * sf + sidx[q]]);
        k3 = u[TRK * sf + sidx[q]] / 3.0;
      }
      bs.set(q, p, e, k3);
    }
  }

  // this thread's point
  const int lx = t % TX, ly = (t / TX) % TY, lz = t / (TX * TY);
  const int c0 = (lz + M) * B::X * B::Y + (ly + M) * B::X + (lx + M);
  const double ih[3] = {1.0 / A.h[0], 1.0 / A.h[1], 1.0 / A.h[2]};

  // per component: the value, first derivatives of g and K; the second
  // derivatives of g go straight into the Riemann pair components R[P][Q]
  // (their part (d_j d_k g_il + d_i d_l g_jk - d_i d_k g_jl - d_j d_l g_ik)/2)
  Acc a;
#pragma unroll
  for (int P = 0; P < 3; ++P)
#pragma unroll
    for (int Q = 0; Q < 3; ++Q) a.R[P][Q] = 0.0;
  component<ORDER, 0>(a, u, sf, sidx, t, c0, ih, bs, gs, ks);
  component<ORDER, 1>(a, u, sf, sidx, t, c0, ih, bs, gs, ks);
  component<ORDER, 2>(a, u, sf, sidx, t, c0, ih, bs, gs, ks);
  component<ORDER, 3>(a, u, sf, sidx, t, c0, ih, bs, gs, ks);
  component<ORDER, 4>(a, u, sf, sidx, t, c0, ih, bs, gs, ks);
  component<ORDER, 5>(a, u, sf, sidx, t, c0, ih, bs, gs, ks);
  const double(&gm)[6] = a.gm;
  const double(&K)[6] = a.K;
  const double(&dg)[3][6] = a.dg;
  const double(&dK)[3][6] = a.dK;
  double(&R)[3][3] = a.R;


  const int ix = tx0 + lx, iy = ty0 + ly, iz = tz0 + lz;
  if (ix >= A.n[0] || iy >= A.n[1] || iz >= A.n[2]) return;

  // inverse metric (adjugate over determinant) and sqrt(det g)
  const double det = gm[0] * (gm[3] * gm[5] - gm[4] * gm[4]) -
                     gm[1] * (gm[1] * gm[5] - gm[4] * gm[2]) +
                     gm[2] * (gm[1] * gm[4] - gm[3] * gm[2]);
  const double idet = 1.0 / det;
  double gu[6];
  gu[0] = (gm[3] * gm[5] - gm[4] * gm[4]) * idet;
  gu[1] = (gm[2] * gm[4] - gm[1] * gm[5]) * idet;
  gu[2] = (gm[1] * gm[4] - gm[2] * gm[3]) * idet;
  gu[3] = (gm[0] * gm[5] - gm[2] * gm[2]) * idet;
  gu[4] = (gm[1] * gm[2] - gm[0] * gm[4]) * idet;
  gu[5] = (gm[0] * gm[3] - gm[1] * gm[1]) * idet;
  const double sdet = sqrt(det);

  // Christoffel symbols: first kind Gl[k][ij] = (d_i g_kj + d_j g_ki -
  // d_k g_ij)/2, second kind Gu[m][ij] = g^mk Gl[k][ij]
  double Gl[3][6], Gu[3][6];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j)
        Gl[k][sy6(i, j)] =
            0.5 * (dg[i][sy6(k, j)] + dg[j][sy6(k, i)] - dg[k][sy6(i, j)]);
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int ij = 0; ij < 6; ++ij)
      Gu[m][ij] = gu[sy6(m, 0)] * Gl[0][ij] + gu[sy6(m, 1)] * Gl[1][ij] +
                  gu[sy6(m, 2)] * Gl[2][ij];

  // the rest of the spatial Riemann projection over index pairs
  // P = (i, j), Q = (k, l):
  //   R_ijkl = (second derivatives, above)
  //          + Gl_n,jk Gu^n_il - Gl_n,jl Gu^n_ik + K_ik K_jl - K_il K_jk
#pragma unroll
  for (int P = 0; P < 3; ++P)
#pragma unroll
    for (int Q = P; Q < 3; ++Q) {
      const int i = PI[P], j = PJ[P], k = PI[Q], l = PJ[Q];
      double r = R[P][Q];
#pragma unroll
      for (int n = 0; n < 3; ++n)
        r += Gl[n][sy6(j, k)] * Gu[n][sy6(i, l)] -
             Gl[n][sy6(j, l)] * Gu[n][sy6(i, k)];
      r += K[sy6(i, k)] * K[sy6(j, l)] - K[sy6(i, l)] * K[sy6(j, k)];
      R[P][Q] = r;
      R[Q][P] = r;
    }
  // electric part E_jl = g^ik R_ijkl (= R_ujul)
  double E[6];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int l = j; l < 3; ++l) {
      double e = 0.0;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) e += gu[sy6(i, k)] * rpair(R, i, j, k, l);
      E[sy6(j, l)] = e;
    }

  // the triad at the point (coordinates relative to the centre)
  const double x = A.origin[0] + ix * A.h[0] - A.centre[0];
  const double y = A.origin[1] + iy * A.h[1] - A.centre[1];
  const double z = A.origin[2] + iz * A.h[2] - A.centre[2];
  double ph[3] = {-y, x, 0.0};
  double rr[3] = {x, y, z};
  const double cr[3] = {ph[1] * rr[2] - ph[2] * rr[1],
                        ph[2] * rr[0] - ph[0] * rr[2],
                        ph[0] * rr[1] - ph[1] * rr[0]};
  double th[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
    th[i] = sdet * (gu[sy6(i, 0)] * cr[0] + gu[sy6(i, 1)] * cr[1] +
                    gu[sy6(i, 2)] * cr[2]);
  {
    const double s = 1.0 / sqrt(gdot(gm, ph, ph));
#pragma unroll
    for (int i = 0; i < 3; ++i) ph[i] *= s;
  }
  {
    const double d = gdot(gm, rr, ph);
#pragma unroll
    for (int i = 0; i < 3; ++i) rr[i] -= d * ph[i];
    const double s = 1.0 / sqrt(gdot(gm, rr, rr));
#pragma unroll
    for (int i = 0; i < 3; ++i) rr[i] *= s;
  }
  {
    const double d1 = gdot(gm, th, ph), d2 = gdot(gm, th, rr);
#pragma unroll
    for (int i = 0; i < 3; ++i) th[i] -= d1 * ph[i] + d2 * rr[i];
    const double s = 1.0 / sqrt(gdot(gm, th, th));
#pragma unroll
    for (int i = 0; i < 3; ++i) th[i] *= s;
  }
  // n^i = -rhat^i/sqrt2 (n^u = 1/sqrt2), mb^i = (thetahat^i - i phihat^i)/sqrt2
  constexpr double r2 = 0.70710678118654752440;
  double nv[3];
  C2 mb[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    nv[i] = -r2 * rr[i];
    mb[i] = {r2 * th[i], -r2 * ph[i]};
  }

  // R_ijkl n^i mb^j n^k mb^l = sum_PQ R_PQ B^P B^Q
  C2 Bv[3];
#pragma unroll
  for (int P = 0; P < 3; ++P) {
    const int i = PI[P], j = PJ[P];
    Bv[P] = cadd(cscale(mb[j], nv[i]), cscale(mb[i], -nv[j]));
  }
  C2 psi = {0.0, 0.0};
#pragma unroll
  for (int P = 0; P < 3; ++P)
#pragma unroll
    for (int Q = 0; Q < 3; ++Q)
      psi = cadd(psi, cscale(cmul(Bv[P], Bv[Q]), R[P][Q]));

  // sqrt2 R_ujkl mb^j n^k mb^l with R_ujkl = DK_k,jl - DK_l,jk,
  // DK_k,ij = d_k K_ij - Gu^m_ki K_mj - Gu^m_kj K_im
  C2 t2 = {0.0, 0.0};
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) {
        double d = dK[k][sy6(i, j)];
#pragma unroll
        for (int m = 0; m < 3; ++m)
          d -= Gu[m][sy6(k, i)] * K[sy6(m, j)] + Gu[m][sy6(k, j)] * K[sy6(i, m)];
        // DK_k,ij contributes to R_u i k j (as D_k K_ij with (j, l) = (i, j))
        // and, with k in the last slot, to R_u i j k with a minus sign:
        //   sum_jkl (DK_k,jl - DK_l,jk) mb^j n^k mb^l
        //   = sum_k,(ij) DK_k,ij (mb^i n^k mb^j - mb^i mb^k n^j)
        // (each unordered pair i != j counted twice, by symmetry of DK)
        const C2 a = cscale(cmul(mb[i], mb[j]), nv[k]);
        const C2 b1 = cscale(cmul(mb[i], mb[k]), nv[j]);
        const C2 b2 = cscale(cmul(mb[j], mb[k]), nv[i]);
        C2 w;
        if (i == j)
          w = cadd(a, cscale(b1, -1.0));
        else
          w = cadd(cscale(a, 2.0), cscale(cadd(b1, b2), -1.0));
        t2 = cadd(t2, cscale(w, d));
      }
  psi = cadd(psi, cscale(t2, 2.0 * r2));

  // (1/2) E_jl mb^j mb^l
  C2 t3 = {0.0, 0.0};
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int l = 0; l < 3; ++l)
      t3 = cadd(t3, cscale(cmul(mb[j], mb[l]), E[sy6(j, l)]));
  psi = cadd(psi, cscale(t3, 0.5));

  const int64_t o = int64_t(iz + g) * A.sz + int64_t(iy + g) * A.sy + ix + g;
  A.out[o] = psi.re;
  A.out[sf + o] = psi.im;
}

}  // namespace

hipError_t launch_psi4(const Psi4Args& A, int order, hipStream_t st) {
  const int64_t ntile = int64_t((A.n[0] + TX - 1) / TX) *
                        ((A.n[1] + TY - 1) / TY) * ((A.n[2] + TZ - 1) / TZ);
  const int64_t nblk = 8 * ((ntile + 7) / 8);
  if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
  if (order == 8)
    hipLaunchKernelGGL(k_psi4<8>, dim3(unsigned(nblk)), dim3(256), 0, st, A);
  else
    hipLaunchKernelGGL(k_psi4<4>, dim3(unsigned(nblk)), dim3(256), 0, st, A);
  return hipGetLastError();
}

}  // namespace bssn
