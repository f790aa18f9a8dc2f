// bssn_constraints.hip -- Hamiltonian, momentum and conformal-connection
// constraints in FP64, with deterministic norms.
//
// H = R - K^i_j K^j_i + K^2 and M_i = D_j K^j_i - D_i K (vacuum; Einstein
// Toolkit paper, "Other analysis modules") written in the BSSN variables
// under the algebraic conditions det gt = 1 and tr A~ = 0:
//   R   = e^{-4phi} gt^ij (R~_ij + R^phi_ij)
//       = e^{-4phi} (gt^ij R~_ij - 8 gt^ij D~_i D~_j phi - 8 gt^ij d_i phi d_j phi)
//   H   = R + 2/3 K^2 - A~_ij A~^ij
//   M_i = Gd^k A~_ik + gt^jk d_j A~_ik + Gamma~^j_jk A~^k_i
//         - Gamma~^k_ji A~^j_k + 6 A~^k_i d_k phi - 2/3 d_i K
//   G^i = Gt^i - gt^jk Gamma~^i_jk
// Norms: every workgroup reduces its points (wave shuffles, then LDS) to 8
// partials; one workgroup then folds the partials in a fixed order, so the
// result does not depend on scheduling.
#include <hip/hip_runtime.h>

#include <mutex>

#include "bssn_api_internal.h"
#include "bssn_kernels.h"
#include "bssn_stage.h"

namespace bssn {

template <int ORDER, class L>
__device__ __forceinline__ void grad(const L& ld, int s, const double (&ih)[3],
                                     double (&d1)[3]) {
  using F = FD<ORDER>;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double s1 = 0.0;
#pragma unroll
    for (int k = 1; k <= F::M; ++k)
      s1 += F::a(k) * (ld.ax(s, a, k) - ld.ax(s, a, -k));
    d1[a] = s1 * ih[a];
  }
}

// full symmetric Hessian (S-indexed)
template <int ORDER, class L>
__device__ __forceinline__ void hess(const L& ld, int s, const double (&ih)[3],
                                     double (&dd)[6]) {
  using F = FD<ORDER>;
  const double c0 = ld.c(s);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double s2 = 0.0;
#pragma unroll
    for (int k = 1; k <= F::M; ++k)
      s2 += F::b(k) * ((ld.ax(s, a, k) - c0) + (ld.ax(s, a, -k) - c0));
    dd[S(a, a)] = s2 * ih[a] * ih[a];
  }
  dd[1] = mixed<ORDER, double>(ld, s, 0, 1, ih[0] * ih[1]);
  dd[2] = mixed<ORDER, double>(ld, s, 0, 2, ih[0] * ih[2]);
  dd[4] = mixed<ORDER, double>(ld, s, 1, 2, ih[1] * ih[2]);
}

template <int ORDER, class L>
__device__ __forceinline__ void constraints_point(const L& ld,
                                                  const double (&ih)[3],
                                                  double& H, double (&M)[3],
                                                  double (&Gc)[3]) {
  double gt[6], At[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    gt[m] = ld.c(GXX + m);
    At[m] = ld.c(AXX + m);
  }
  const double c00 = gt[3] * gt[5] - gt[4] * gt[4];
  const double c01 = gt[2] * gt[4] - gt[1] * gt[5];
  const double c02 = gt[1] * gt[4] - gt[2] * gt[3];
  const double idet = 1.0 / (gt[0] * c00 + gt[1] * c01 + gt[2] * c02);
  double gu[6];
  gu[0] = c00 * idet;
  gu[1] = c01 * idet;
  gu[2] = c02 * idet;
  gu[3] = (gt[0] * gt[5] - gt[2] * gt[2]) * idet;
  gu[4] = (gt[1] * gt[2] - gt[0] * gt[4]) * idet;
  gu[5] = (gt[0] * gt[3] - gt[1] * gt[1]) * idet;
  double Aud[3][3], Auu[6];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      Aud[i][j] = gu[S(i, 0)] * At[S(0, j)] + gu[S(i, 1)] * At[S(1, j)] +
                  gu[S(i, 2)] * At[S(2, j)];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j)
      Auu[S(i, j)] = Aud[i][0] * gu[S(0, j)] + Aud[i][1] * gu[S(1, j)] +
                     Aud[i][2] * gu[S(2, j)];
  const double AA = At[0] * Auu[0] + At[3] * Auu[3] + At[5] * Auu[5] +
                    2.0 * (At[1] * Auu[1] + At[2] * Auu[2] + At[4] * Auu[4]);

  double dgt[6][3], trR = 0.0;
  double Rt[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    BSSN_PHASE();
    grad<ORDER>(ld, GXX + m, ih, dgt[m]);
    double dd[6];
    hess<ORDER>(ld, GXX + m, ih, dd);
    Rt[m] = -0.5 * (gu[0] * dd[0] + gu[3] * dd[3] + gu[5] * dd[5] +
                    2.0 * (gu[1] * dd[1] + gu[2] * dd[2] + gu[4] * dd[4]));
    keep(Rt[m]);
#pragma unroll
    for (int a = 0; a < 3; ++a) keep(dgt[m][a]);
  }
  double Gl[3][6], Gu[3][6];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = j; k < 3; ++k)
        Gl[i][S(j, k)] =
            0.5 * (dgt[S(i, j)][k] + dgt[S(i, k)][j] - dgt[S(j, k)][i]);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int m = 0; m < 6; ++m)
      Gu[i][m] = gu[S(i, 0)] * Gl[0][m] + gu[S(i, 1)] * Gl[1][m] +
                 gu[S(i, 2)] * Gl[2][m];
  double Gd[3];
  {
    double Q[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      double s = 0.0;
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
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        s -= 0.5 * (Gl[i][S(j, k)] + Gl[j][S(i, k)]) * Gd[k];
#pragma unroll
        for (int l = 0; l < 3; ++l)
#pragma unroll
          for (int m = 0; m < 3; ++m)
            s += gu[S(l, m)] * (Gu[k][S(l, i)] * Gl[j][S(k, m)] +
                                Gu[k][S(l, j)] * Gl[i][S(k, m)] +
                                Gu[k][S(i, m)] * Gl[k][S(l, j)]);
      }
      Rt[S(i, j)] += s;
    }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    BSSN_PHASE();
    double dG[3];
    grad<ORDER>(ld, GAMX + k, ih, dG);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j)
        Rt[S(i, j)] += 0.5 * (gt[S(k, i)] * dG[j] + gt[S(k, j)] * dG[i]);
  }
#pragma unroll
  for (int m = 0; m < 6; ++m) keep(Rt[m]);
  trR = gu[0] * Rt[0] + gu[3] * Rt[3] + gu[5] * Rt[5] +
        2.0 * (gu[1] * Rt[1] + gu[2] * Rt[2] + gu[4] * Rt[4]);

  BSSN_PHASE();
  double dphi[3], ddphi[6];
  grad<ORDER>(ld, PHI, ih, dphi);
  hess<ORDER>(ld, PHI, ih, ddphi);
  double trDD = 0.0, dphi2 = 0.0;
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    const double DD = ddphi[m] - (Gu[0][m] * dphi[0] + Gu[1][m] * dphi[1] +
                                  Gu[2][m] * dphi[2]);
    const double w = (m == 0 || m == 3 || m == 5) ? 1.0 : 2.0;
    trDD += w * gu[m] * DD;
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) dphi2 += gu[S(i, j)] * dphi[i] * dphi[j];
  const double phi = ld.c(PHI), trK = ld.c(TRK);
  const double R = exp(-4.0 * phi) * (trR - 8.0 * trDD - 8.0 * dphi2);
  H = R + (2.0 / 3.0) * trK * trK - AA;

  BSSN_PHASE();
  double dK[3];
  grad<ORDER>(ld, TRK, ih, dK);
#pragma unroll
  for (int i = 0; i < 3; ++i) M[i] = -(2.0 / 3.0) * dK[i];
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    BSSN_PHASE();
    double dA[3];
    grad<ORDER>(ld, AXX + m, ih, dA);
    // gt^jk d_j A~_ik: slot m = S(i,k) contributes to M_i and (i != k) M_k
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (S(i, k) == m)
          M[i] += gu[S(0, k)] * dA[0] + gu[S(1, k)] * dA[1] +
                  gu[S(2, k)] * dA[2];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      s += Gd[k] * At[S(i, k)] + 6.0 * Aud[k][i] * dphi[k];
#pragma unroll
      for (int j = 0; j < 3; ++j)
        s += Gu[j][S(j, k)] * Aud[k][i] - Gu[k][S(j, i)] * Aud[j][k];
    }
    M[i] += s;
    const double c = gu[0] * Gu[i][0] + gu[3] * Gu[i][3] + gu[5] * Gu[i][5] +
                     2.0 * (gu[1] * Gu[i][1] + gu[2] * Gu[i][2] +
                            gu[4] * Gu[i][4]);
    Gc[i] = ld.c(GAMX + i) - c;
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// partial order: 0 sum H^2, 1 max|H|, 2 sum|M|^2, 3 max|M|, 4 sum|G|^2,
// 5 max|G|, 6 used, 7 non-finite
template <int ORDER, bool PERIODIC>
__global__ void __launch_bounds__(256)
    k_constraints(const ConstraintArgs A, double* __restrict__ partials) {
  constexpr int R = FD<ORDER>::R;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  const bool active = x < A.n[0] && y < A.n[1];
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (active) {
    const int g = A.ghost;
    const int32_t nbytes = int32_t(A.sf * 8);
    const uint32_t sy8 = uint32_t(A.sy) * 8u, sz8 = uint32_t(A.sz) * 8u;
    const uint32_t vc =
        uint32_t(z + g) * sz8 + uint32_t(y + g) * sy8 + uint32_t(x + g) * 8u;
    const double ih[3] = {1.0 / A.h[0], 1.0 / A.h[1], 1.0 / A.h[2]};
    double H, M[3], Gc[3];
    if constexpr (!PERIODIC) {
      LdStatic<R> ld;
      ld.u = A.u;
      ld.sf = A.sf;
      ld.nbytes = nbytes;
      ld.vlo = vc - uint32_t(R) * (8u + sy8 + sz8);
      ld.str[0] = 8u;
      ld.str[1] = sy8;
      ld.str[2] = sz8;
      constraints_point<ORDER>(ld, ih, H, M, Gc);
    } else {
      LdPeriodic<R> ld;
      ld.u = A.u;
      ld.sf = A.sf;
      ld.nbytes = nbytes;
      const int pos[3] = {x, y, z};
      const uint32_t st[3] = {8u, sy8, sz8};
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int k = -R; k <= R; ++k) {
          int q = pos[a] + k;
          q = q < 0 ? q + A.n[a] : (q >= A.n[a] ? q - A.n[a] : q);
          ld.o[a][R + k] = uint32_t(q + g) * st[a];
        }
      constraints_point<ORDER>(ld, ih, H, M, Gc);
    }
    if (A.H) bstore(rsrc(A.H, nbytes), vc, H);
    if (A.M)
      for (int i = 0; i < 3; ++i) bstore(rsrc(A.M + i * A.sf, nbytes), vc, M[i]);
    if (A.Gc)
      for (int i = 0; i < 3; ++i)
        bstore(rsrc(A.Gc + i * A.sf, nbytes), vc, Gc[i]);
    bool use = true;
    const double xc = A.origin[0] + x * A.h[0], yc = A.origin[1] + y * A.h[1],
                 zc = A.origin[2] + z * A.h[2];
    for (int c = 0; c < A.ncent; ++c) {
      const double dx = xc - A.centres[c][0], dy = yc - A.centres[c][1],
                   dz = zc - A.centres[c][2];
      if (sqrt(dx * dx + dy * dy + dz * dz) <= A.r_exc) use = false;
    }
    if (use) {
      const double m2 = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
      const double g2 = Gc[0] * Gc[0] + Gc[1] * Gc[1] + Gc[2] * Gc[2];
      const double mm = sqrt(m2), gm = sqrt(g2);
      if (!isfinite(H) || !isfinite(mm) || !isfinite(gm)) {
        v[7] = 1.0;
      } else {
        v[0] = H * H;
        v[1] = fabs(H);
        v[2] = mm * mm;
        v[3] = mm;
        v[4] = gm * gm;
        v[5] = gm;
        v[6] = 1.0;
      }
    }
  }
  __shared__ double red[8][16];
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  const int nw = (blockDim.x * blockDim.y + 63) >> 6;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const bool mx = (k == 1 || k == 3 || k == 5);
    const double w = mx ? wave_max(v[k]) : wave_sum(v[k]);
    if ((tid & 63) == 0) red[k][tid >> 6] = w;
  }
  __syncthreads();
  if (tid < 8) {
    const bool mx = (tid == 1 || tid == 3 || tid == 5);
    double acc = red[tid][0];
    for (int w = 1; w < nw; ++w)
      acc = mx ? fmax(acc, red[tid][w]) : acc + red[tid][w];
    const size_t b =
        blockIdx.x + gridDim.x * (blockIdx.y + size_t(gridDim.y) * blockIdx.z);
    partials[b * 8 + tid] = acc;
  }
}

// One workgroup folds nb partial records in a fixed order.
__global__ void __launch_bounds__(256)
    k_norms(const double* __restrict__ partials, long nb,
            double* __restrict__ norms) {
  __shared__ double red[8][256];
  const int t = threadIdx.x;
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (long b = t; b < nb; b += 256)
    for (int k = 0; k < 8; ++k) {
      const double p = partials[b * 8 + k];
      v[k] = (k == 1 || k == 3 || k == 5) ? fmax(v[k], p) : v[k] + p;
    }
  for (int k = 0; k < 8; ++k) red[k][t] = v[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w)
      for (int k = 0; k < 8; ++k)
        red[k][t] = (k == 1 || k == 3 || k == 5)
                        ? fmax(red[k][t], red[k][t + w])
                        : red[k][t] + red[k][t + w];
    __syncthreads();
  }
  if (t == 0) {
    const double n = red[6][0];
    norms[0] = n > 0 ? sqrt(red[0][0] / n) : 0.0;
    norms[1] = red[1][0];
    norms[2] = n > 0 ? sqrt(red[2][0] / n) : 0.0;
    norms[3] = red[3][0];
    norms[4] = n > 0 ? sqrt(red[4][0] / n) : 0.0;
    norms[5] = red[5][0];
    norms[6] = n;
    norms[7] = red[7][0];
  }
}

static void cgrid(const ConstraintArgs& A, dim3& grd, dim3& blk) {
  const int bx = A.n[0] > 32 ? 64 : 32;
  blk = dim3(bx, 256 / bx, 1);
  grd = dim3((A.n[0] + bx - 1) / bx, (A.n[1] + blk.y - 1) / blk.y, A.n[2]);
}

int constraint_blocks(const ConstraintArgs& A) {
  dim3 g, b;
  cgrid(A, g, b);
  return int(g.x * g.y * g.z);
}

hipError_t launch_constraints(const ConstraintArgs& A, int order,
                              double* partials, int nblocks_max,
                              double* norms, hipStream_t st) {
  dim3 grd, blk;
  cgrid(A, grd, blk);
  const long nb = long(grd.x) * grd.y * grd.z;
  if (nb > nblocks_max) return hipErrorInvalidValue;
  if (order == 4) {
    if (A.periodic)
      hipLaunchKernelGGL((k_constraints<4, true>), grd, blk, 0, st, A, partials);
    else
      hipLaunchKernelGGL((k_constraints<4, false>), grd, blk, 0, st, A, partials);
  } else {
    if (A.periodic)
      hipLaunchKernelGGL((k_constraints<8, true>), grd, blk, 0, st, A, partials);
    else
      hipLaunchKernelGGL((k_constraints<8, false>), grd, blk, 0, st, A, partials);
  }
  hipLaunchKernelGGL(k_norms, dim3(1), dim3(256), 0, st, partials, nb, norms);
  return hipGetLastError();
}

// ---- mixed-precision routing statistics ----------------------------------------
__global__ void __launch_bounds__(256)
    k_tile_count(const Patch P, const double thr,
                 unsigned long long* __restrict__ counter) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  const bool active = x < P.n[0] && y < P.n[1];
  const int g = P.ghost;
  const uint32_t vc = uint32_t(z + g) * uint32_t(P.sz) * 8u +
                      uint32_t(y + g) * uint32_t(P.sy) * 8u +
                      uint32_t(x + g) * 8u;
  const bool f64 = tile_needs_fp64(P, active, vc, int32_t(P.sf * 8), thr);
  if (threadIdx.x == 0 && threadIdx.y == 0 && f64) atomicAdd(counter, 1ull);
}

// The same predicate over the LDS kernel's 16 x 4 x 4 tiles (one block per
// tile, thread = point as in that kernel).
__global__ void __launch_bounds__(256)
    k_tile_count_lds(const Patch P, const double thr, const int ntx,
                     const int nty, unsigned long long* __restrict__ counter) {
  const int t = blockIdx.x, tid = threadIdx.x;
  const int ix = t % ntx, iy = (t / ntx) % nty, iz = t / (ntx * nty);
  const int x = ix * kLdsTile[0] + (tid & 15);
  const int y = iy * kLdsTile[1] + ((tid >> 4) & 3);
  const int z = iz * kLdsTile[2] + (tid >> 6);
  const bool active = x < P.n[0] && y < P.n[1] && z < P.n[2];
  const int g = P.ghost;
  const uint32_t vc = uint32_t(z + g) * uint32_t(P.sz) * 8u +
                      uint32_t(y + g) * uint32_t(P.sy) * 8u +
                      uint32_t(x + g) * 8u;
  const bool f64 = tile_needs_fp64(P, active, vc, int32_t(P.sf * 8), thr);
  if (tid == 0 && f64) atomicAdd(counter, 1ull);
}

void tile_grid(const Patch& P, int lds, dim3& grd, dim3& blk) {
  if (lds) {
    const int ntx = (P.n[0] + kLdsTile[0] - 1) / kLdsTile[0];
    const int nty = (P.n[1] + kLdsTile[1] - 1) / kLdsTile[1];
    const int ntz = (P.n[2] + kLdsTile[2] - 1) / kLdsTile[2];
    grd = dim3(ntx * nty * ntz, 1, 1);
    blk = dim3(256, 1, 1);
    return;
  }
  stage_tile_shape(P, 0, blk);
  grd = dim3((P.n[0] + blk.x - 1) / blk.x, (P.n[1] + blk.y - 1) / blk.y,
             P.n[2]);
}

hipError_t launch_tile_count(const Patch& P, double thr, int lds,
                             unsigned long long* counter, hipStream_t st) {
  dim3 grd, blk;
  tile_grid(P, lds, grd, blk);
  if (lds) {
    const int ntx = (P.n[0] + kLdsTile[0] - 1) / kLdsTile[0];
    const int nty = (P.n[1] + kLdsTile[1] - 1) / kLdsTile[1];
    hipLaunchKernelGGL(k_tile_count_lds, grd, blk, 0, st, P, thr, ntx, nty,
                       counter);
  } else {
    hipLaunchKernelGGL(k_tile_count, grd, blk, 0, st, P, thr, counter);
  }
  return hipGetLastError();
}

}  // namespace bssn

// ---- constraints without allocation ---------------------------------------------
// The per-block partial norms of bssn_constraints_noalloc live in this
// file-scope device array: kNoAllocRecords records of 8 doubles (16 MiB),
// which covers grids of up to 262,144 constraint blocks (a 384^3 grid needs
// 221,184).  Each GPU holds its own copy for the life of the process.  Host
// code never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): it uses the device address that
// hipGetSymbolAddress returns, once per device, with that device current.
namespace bssn {
constexpr int kNoAllocRecords = 1 << 18;
static __device__ __align__(256) double scratch[size_t(kNoAllocRecords) * 8];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (set up on the first
// call on the device).
int scratch_address(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(BSSN_EUNSUPPORTED, "device %d beyond the %d the library "
                "tracks", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return BSSN_OK;
}
}  // namespace
}  // namespace bssn

extern "C" int bssn_constraints_noalloc(const bssn_grid* grid,
                                        const bssn_params* params,
                                        const double* u, double* H,
                                        double* M, double* G,
                                        const double* centres, int ncent,
                                        double r_exc, double* norms,
                                        void* stream) {
  using namespace bssn;
  ConstraintArgs A{};
  int rc = constraint_args(grid, params, u, H, M, G, centres, ncent, r_exc,
                           norms, &A);
  if (rc) return rc;
  const long nb = constraint_blocks(A);
  if (nb > kNoAllocRecords)
    return fail(BSSN_EINVAL, "the grid needs %ld partial records; the "
                "allocation-free constraints hold at most %d (a 384^3 grid "
                "needs 221184)", nb, kNoAllocRecords);
  double* part = nullptr;
  if ((rc = scratch_address(&part))) return rc;
  // every record a launch reads is written by the same launch: nothing to
  // clear
  const hipError_t e = launch_constraints(A, params->fd_order, part,
                                          kNoAllocRecords, norms,
                                          (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "bssn_constraints_noalloc launch");
  return BSSN_OK;
}
