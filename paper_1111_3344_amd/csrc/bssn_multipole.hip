// bssn_multipole.hip -- multipole coefficients of a complex grid function on
// a coordinate sphere (Einstein Toolkit paper, analysis section: the
// multipole module projects a field interpolated onto spheres onto
// spin-weighted spherical harmonics, C^lm = integral conj(sY_lm) u r^2 dOmega).
//
// Four launches:
//   k_gl_nodes      Gauss-Legendre nodes and weights in cos(theta), by Newton
//                   iteration on the Legendre recurrence (one thread per node);
//   k_sphere_interp one thread per sphere point (theta_j, phi_k): the
//                   tricubic interpolation of the real and imaginary parts
//                   (4 x 4 x 4 storage points, block clamped into the grid);
//   k_multipole     one workgroup per (l, m, chunk of the points): the sum
//                   of conj(sY_lm) u w_j (2 pi / n_phi) over its points, a
//                   fixed-order tree reduction;
//   k_multipole_sum one thread per (l, m): the chunks added in order (the
//                   result is deterministic), times r^2.
// sY_lm (Goldberg's sum) is evaluated with half-angle powers,
//   sin^{2l-k}(theta/2) cos^{k}(theta/2), k = 2r + s - m in [0, 2l],
// so no cotangent is formed.
#include <hip/hip_runtime.h>

#include "bssn_internal.h"
#include "bssn_kernels.h"

namespace bssn {
namespace {

__device__ __forceinline__ double ipow(double x, int n) {
  double r = 1.0;
  while (n > 0) {
    if (n & 1) r *= x;
    x *= x;
    n >>= 1;
  }
  return r;
}

__device__ __forceinline__ double fact(int n) {
  double r = 1.0;
  for (int k = 2; k <= n; ++k) r *= k;
  return r;
}

__device__ __forceinline__ double binom(int n, int k) {
  if (k < 0 || k > n) return 0.0;
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// Nodes ascending in x = cos(theta).
__global__ void __launch_bounds__(64)
    k_gl_nodes(const int n, double* __restrict__ x, double* __restrict__ w) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int jd = n - 1 - j;  // the guess below is descending in j
  double z = cos(M_PI * (jd + 0.75) / (n + 0.5));
  double dp = 1.0;
  for (int it = 0; it < 100; ++it) {
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    if (n == 1) p0 = 1.0;
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    const double dz = p1 / dp;
    z -= dz;
    if (fabs(dz) <= 1e-15 * fabs(z)) break;  // dz = 0 at the middle node
  }
  // the weight from the derivative at the converged node
  double p0 = 1.0, p1 = z;
  for (int k = 2; k <= n; ++k) {
    const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  dp = n * (z * p1 - p0) / (z * z - 1.0);
  x[j] = z;
  w[j] = 2.0 / ((1.0 - z * z) * dp * dp);
}

__global__ void __launch_bounds__(64)
    k_sphere_interp(const MultipoleArgs A, const double* __restrict__ x,
                    double* __restrict__ val) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= A.ntheta * A.nphi) return;
  const int j = p / A.nphi, k = p % A.nphi;
  const double ct = x[j], st = sqrt(fmax(0.0, 1.0 - ct * ct));
  const double ph = 2.0 * M_PI * k / A.nphi;
  const double pos[3] = {A.centre[0] + A.radius * st * cos(ph),
                         A.centre[1] + A.radius * st * sin(ph),
                         A.centre[2] + A.radius * ct};
  const int g = A.ghost;
  double wt[3][4];
  int b[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int N = A.n[a] + 2 * g;
    const double s = (pos[a] - (A.origin[a] - g * A.h[a])) / A.h[a];
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
      wt[a][m] = q;
    }
  }
  double re = 0.0, im = 0.0;
  const int64_t base = int64_t(b[2]) * A.sz + int64_t(b[1]) * A.sy + b[0];
  for (int kk = 0; kk < 4; ++kk)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj)
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        const double w = wt[2][kk] * wt[1][jj] * wt[0][ii];
        const int64_t o = base + kk * A.sz + jj * A.sy + ii;
        re += w * A.re[o];
        if (A.im) im += w * A.im[o];
      }
  val[2 * p] = re;
  val[2 * p + 1] = im;
}

__global__ void __launch_bounds__(256)
    k_multipole(const MultipoleArgs A, const double* __restrict__ x,
                const double* __restrict__ w, const double* __restrict__ val,
                const int nchunk, double* __restrict__ part) {
  __shared__ double sre[256], sim[256];
  const int q = blockIdx.x / nchunk, chunk = blockIdx.x % nchunk;
  int l = 0;
  while ((l + 1) * (l + 1) <= q) ++l;
  const int m = q - l * l - l;
  const int s = A.spin;
  double are = 0.0, aim = 0.0;
  if (l >= (s < 0 ? -s : s)) {
    const double pre =
        ((m & 1) ? -1.0 : 1.0) *
        sqrt(fact(l + m) * fact(l - m) * (2 * l + 1) /
             (4.0 * M_PI * fact(l + s) * fact(l - s)));
    const double dphi = 2.0 * M_PI / A.nphi;
    const int npts = A.ntheta * A.nphi;
    for (int p = chunk * 256 + threadIdx.x; p < npts; p += nchunk * 256) {
      const int j = p / A.nphi, k = p % A.nphi;
      const double ct = x[j];
      const double sh = sqrt(fmax(0.0, 0.5 * (1.0 - ct)));
      const double ch = sqrt(fmax(0.0, 0.5 * (1.0 + ct)));
      double sum = 0.0;
      for (int r = 0; r <= l - s; ++r) {
        const int kb = r + s - m;
        if (kb < 0 || kb > l + s) continue;
        const int e = 2 * r + s - m;  // cot power, in [0, 2l]
        const double sign = ((l - r - s) & 1) ? -1.0 : 1.0;
        sum += sign * binom(l - s, r) * binom(l + s, kb) *
               ipow(sh, 2 * l - e) * ipow(ch, e);
      }
      const double y = pre * sum;  // real part of sY_lm without e^{i m phi}
      double sn, cs;
      sincos(m * (dphi * k), &sn, &cs);
      // conj(Y) u = y (cos - i sin)(u_re + i u_im)
      const double ur = val[2 * p], ui = val[2 * p + 1];
      const double wq = w[j] * dphi;
      are += wq * y * (cs * ur + sn * ui);
      aim += wq * y * (cs * ui - sn * ur);
    }
  }
  sre[threadIdx.x] = are;
  sim[threadIdx.x] = aim;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      sre[threadIdx.x] += sre[threadIdx.x + h];
      sim[threadIdx.x] += sim[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * (q * nchunk + chunk)] = sre[0];
    part[2 * (q * nchunk + chunk) + 1] = sim[0];
  }
}

// One thread per (l, m): the chunks' partial sums added in chunk order.
__global__ void __launch_bounds__(64)
    k_multipole_sum(const int nq, const int nchunk, const double radius,
                    const double* __restrict__ part,
                    double* __restrict__ coeffs) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  double re = 0.0, im = 0.0;
  for (int c = 0; c < nchunk; ++c) {
    re += part[2 * (q * nchunk + c)];
    im += part[2 * (q * nchunk + c) + 1];
  }
  coeffs[2 * q] = re * radius * radius;
  coeffs[2 * q + 1] = im * radius * radius;
}

}  // namespace

hipError_t launch_multipole(const MultipoleArgs& A, double* work,
                            double* coeffs, hipStream_t st) {
  double* x = work;
  double* w = work + A.ntheta;
  double* val = work + 2 * A.ntheta;
  hipLaunchKernelGGL(k_gl_nodes, dim3((A.ntheta + 63) / 64), dim3(64), 0, st,
                     A.ntheta, x, w);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int npts = A.ntheta * A.nphi;
  hipLaunchKernelGGL(k_sphere_interp, dim3((npts + 63) / 64), dim3(64), 0, st,
                     A, x, val);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nq = (A.lmax + 1) * (A.lmax + 1);
  const int nchunk = multipole_chunks(A.ntheta, A.nphi);
  double* part = val + 2 * int64_t(npts);
  hipLaunchKernelGGL(k_multipole, dim3(nq * nchunk), dim3(256), 0, st, A, x,
                     w, val, nchunk, part);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_multipole_sum, dim3((nq + 63) / 64), dim3(64), 0, st,
                     nq, nchunk, A.radius, part, coeffs);
  return hipGetLastError();
}

}  // namespace bssn
