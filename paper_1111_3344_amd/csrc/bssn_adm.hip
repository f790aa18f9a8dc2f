// bssn_adm.hip -- initial conversion from the ADM variables to the BSSN
// state (Einstein Toolkit paper, spacetime curvature evolution, initial
// conditions).
//
// Three passes:
//   1. every storage point: phi = ln(det g)/12, gt_ij = e^{-4 phi} g_ij,
//      K = g^ij K_ij, At_ij = e^{-4 phi}(K_ij - g_ij K/3), alpha and beta^i
//      copied, B^i = 0 and the lapse time-derivative slot 0;
//   2. interior points: Gt^i = gt^ij gt^kl Gt_jkl with
//      Gt_jkl = (d_l gt_jk + d_k gt_jl - d_j gt_kl)/2, the derivatives
//      centred differences of the grid's order (pairwise form) of the
//      converted metric;
//   3. ghost layers, innermost first (one launch each): Gt^i by the cubic
//      X(p) = 4X(p-n) - 6X(p-2n) + 4X(p-3n) - X(p-4n) along n, the outward
//      normal of p's face, or the sum of the face normals at an edge or
//      corner.
// Memory-bound (the ADM input, 16 values per point, and the state out).
#include <hip/hip_runtime.h>

#include "bssn_internal.h"
#include "bssn_kernels.h"

namespace bssn {
namespace {

// symmetric pair -> 0..5 (xx xy xz yy yz zz)
__device__ __forceinline__ constexpr int sym(int i, int j) {
  return i > j ? sym(j, i) : (i == 0 ? j : (i == 1 ? 2 + j : 5));
}

__device__ __forceinline__ double det3(const double (&m)[3][3]) {
  return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) -
         m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
         m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
}

// inverse by the adjugate: inv[i][j] = cofactor(j, i) / det
__device__ __forceinline__ void inv3(const double (&m)[3][3],
                                     double (&inv)[3][3]) {
  const double d = det3(m);
  inv[0][0] = (m[1][1] * m[2][2] - m[1][2] * m[2][1]) / d;
  inv[0][1] = -(m[0][1] * m[2][2] - m[0][2] * m[2][1]) / d;
  inv[0][2] = (m[0][1] * m[1][2] - m[0][2] * m[1][1]) / d;
  inv[1][0] = -(m[1][0] * m[2][2] - m[1][2] * m[2][0]) / d;
  inv[1][1] = (m[0][0] * m[2][2] - m[0][2] * m[2][0]) / d;
  inv[1][2] = -(m[0][0] * m[1][2] - m[0][2] * m[1][0]) / d;
  inv[2][0] = (m[1][0] * m[2][1] - m[1][1] * m[2][0]) / d;
  inv[2][1] = -(m[0][0] * m[2][1] - m[0][1] * m[2][0]) / d;
  inv[2][2] = (m[0][0] * m[1][1] - m[0][1] * m[1][0]) / d;
}

__global__ void __launch_bounds__(64) k_adm_point(const AdmArgs A) {
  const int g = A.ghost;
  const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
  if (i >= A.n[0] + 2 * g) return;
  const int64_t idx = int64_t(k) * A.sz + int64_t(j) * A.sy + i;
  double a[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) a[s] = A.adm[int64_t(s) * A.sf + idx];
  double gm[3][3], gu[3][3];
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int q = 0; q < 3; ++q) gm[p][q] = a[sym(p, q)];
  const double phi = log(det3(gm)) / 12.0;
  const double e4 = exp(-4.0 * phi);
  inv3(gm, gu);
  double trK = 0.0;
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int q = 0; q < 3; ++q) trK += gu[p][q] * a[6 + sym(p, q)];
  double* u = A.u + idx;
  const int64_t sf = A.sf;
  u[PHI * sf] = phi;
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    u[(GXX + m) * sf] = e4 * a[m];
    u[(AXX + m) * sf] = e4 * (a[6 + m] - a[m] * trK / 3.0);
  }
  u[TRK * sf] = trK;
  u[ALP * sf] = a[12];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    u[(BETX + d) * sf] = a[13 + d];
    u[(BX + d) * sf] = 0.0;
  }
  u[ADOT * sf] = 0.0;
}

template <int ORDER>
__device__ __forceinline__ double fd_a(int k) {
  if (ORDER == 4) return k == 1 ? 2.0 / 3.0 : -1.0 / 12.0;
  return k == 1 ? 4.0 / 5.0
         : k == 2 ? -1.0 / 5.0
         : k == 3 ? 4.0 / 105.0
                  : -1.0 / 280.0;
}

template <int ORDER>
__global__ void __launch_bounds__(64) k_adm_gamma(const AdmArgs A) {
  constexpr int M = ORDER / 2;
  const int g = A.ghost;
  const int x = blockIdx.x * 64 + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= A.n[0]) return;
  const int64_t idx = int64_t(z + g) * A.sz + int64_t(y + g) * A.sy + x + g;
  const int64_t st[3] = {1, A.sy, A.sz};
  double gt[3][3], gtu[3][3], dg[3][6];
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    const double* v = A.u + (GXX + m) * A.sf + idx;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      double s = 0.0;
#pragma unroll
      for (int kk = 1; kk <= M; ++kk)
        s += fd_a<ORDER>(kk) * (v[kk * st[ax]] - v[-kk * st[ax]]);
      dg[ax][m] = s / A.h[ax];
    }
  }
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int q = 0; q < 3; ++q)
      gt[p][q] = A.u[(GXX + sym(p, q)) * A.sf + idx];
  inv3(gt, gtu);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double G = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int l = 0; l < 3; ++l) {
          const double gl = 0.5 * (dg[l][sym(j, k)] + dg[k][sym(j, l)] -
                                   dg[j][sym(k, l)]);
          G += gtu[i][j] * gtu[k][l] * gl;
        }
    A.u[(GAMX + i) * A.sf + idx] = G;
  }
}

// Layer `layer` of the ghosts: one thread per (point of the layer's shell,
// Gt component), the shell enumerated face by face (z faces whole, y faces
// without their z edges, x faces without either).
__global__ void __launch_bounds__(256)
    k_adm_extrap(const AdmArgs A, const int layer, const int64_t npts) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (t >= npts) return;
  const int ax = A.n[0] + 2 * layer, ay = A.n[1] + 2 * layer,
            az = A.n[2] + 2 * layer;
  int lx, ly, lz;
  const int64_t fz = int64_t(ax) * ay, fy = int64_t(ax) * (az - 2);
  if (t < 2 * fz) {
    const int64_t m = t % fz;
    lz = t < fz ? 0 : az - 1;
    lx = int(m % ax);
    ly = int(m / ax);
  } else if (t < 2 * fz + 2 * fy) {
    const int64_t w = t - 2 * fz, m = w % fy;
    ly = w < fy ? 0 : ay - 1;
    lx = int(m % ax);
    lz = 1 + int(m / ax);
  } else {
    const int64_t fx = int64_t(ay - 2) * (az - 2);
    const int64_t w = t - 2 * fz - 2 * fy, m = w % fx;
    lx = w < fx ? 0 : ax - 1;
    ly = 1 + int(m % (ay - 2));
    lz = 1 + int(m / (ay - 2));
  }
  const int g = A.ghost;
  const int i = lx - layer + g, j = ly - layer + g, k = lz - layer + g;
  const int sx = i < g ? -1 : (i >= A.n[0] + g ? 1 : 0);
  const int sy = j < g ? -1 : (j >= A.n[1] + g ? 1 : 0);
  const int sz = k < g ? -1 : (k >= A.n[2] + g ? 1 : 0);
  double* v = A.u + (GAMX + c) * A.sf;
  const int64_t step = int64_t(sz) * A.sz + int64_t(sy) * A.sy + sx;
  const int64_t p = int64_t(k) * A.sz + int64_t(j) * A.sy + i;
  v[p] = 4.0 * v[p - step] - 6.0 * v[p - 2 * step] + 4.0 * v[p - 3 * step] -
         v[p - 4 * step];
}

// One Euler step of dx/dt = -beta(x) per puncture (object tracking in the
// paper's analysis section), beta by tricubic Lagrange interpolation on the
// 4 x 4 x 4 storage points around x (base node floor((x - x_0)/h) - 1, x_0
// the coordinate of storage index 0, shifted inward to stay in the grid).
__global__ void __launch_bounds__(64)
    k_track(const TrackArgs A, double* __restrict__ pos, const int np,
            const double dt) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const int g = A.ghost;
  double x[3], w[3][4];
  int b[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    x[a] = pos[3 * p + a];
    const int N = A.n[a] + 2 * g;
    const double s = (x[a] - (A.origin[a] - g * A.h[a])) / A.h[a];
    double fs = floor(s);
    if (!(fs >= -2.0)) fs = -2.0;  // also NaN
    if (fs > double(N)) fs = double(N);
    int bb = int(fs) - 1;
    bb = bb < 0 ? 0 : (bb > N - 4 ? N - 4 : bb);
    b[a] = bb;
    const double t = s - bb;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      double q = 1.0;
#pragma unroll
      for (int l = 0; l < 4; ++l)
        if (l != m) q *= (t - l) / double(m - l);
      w[a][m] = q;
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double* f = A.u + (BETX + c) * A.sf;
    double acc = 0.0;
    for (int k = 0; k < 4; ++k)
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          acc += w[2][k] * w[1][j] * w[0][i] *
                 f[int64_t(b[2] + k) * A.sz + int64_t(b[1] + j) * A.sy +
                   (b[0] + i)];
    pos[3 * p + c] = x[c] - dt * acc;
  }
}

}  // namespace

hipError_t launch_track(const TrackArgs& A, double* pos, int np, double dt,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_track, dim3((np + 63) / 64), dim3(64), 0, st, A, pos,
                     np, dt);
  return hipGetLastError();
}

hipError_t launch_from_adm(const AdmArgs& A, hipStream_t st) {
  const int g = A.ghost;
  const dim3 gs((A.n[0] + 2 * g + 63) / 64, A.n[1] + 2 * g, A.n[2] + 2 * g);
  const dim3 gi((A.n[0] + 63) / 64, A.n[1], A.n[2]);
  if (gs.y > 65535u || gs.z > 65535u) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_adm_point, gs, dim3(64), 0, st, A);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (A.order == 8)
    hipLaunchKernelGGL(k_adm_gamma<8>, gi, dim3(64), 0, st, A);
  else
    hipLaunchKernelGGL(k_adm_gamma<4>, gi, dim3(64), 0, st, A);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int layer = 1; layer <= g; ++layer) {
    const int64_t ax = A.n[0] + 2 * layer, ay = A.n[1] + 2 * layer,
                  az = A.n[2] + 2 * layer;
    const int64_t npts = 2 * ax * ay + 2 * ax * (az - 2) +
                         2 * (ay - 2) * (az - 2);
    const int64_t nb = (npts + 255) / 256;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_adm_extrap, dim3(unsigned(nb), 3), dim3(256), 0, st,
                       A, layer, npts);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace bssn
