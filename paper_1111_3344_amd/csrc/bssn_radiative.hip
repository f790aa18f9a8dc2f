// bssn_radiative.hip -- the radiative (Sommerfeld-type) outer boundary: the
// right-hand side on the ghost layers of a static grid (Einstein Toolkit
// paper, spacetime curvature evolution, boundary conditions).
//
// Every evolved component X is taken to be an outgoing spherical wave near
// the boundary, X = X0 + u(r - v0 t)/r, which gives the wave part
//   S = -v0 (x^i d_i X) / r - v0 (X - X0) / r
// with second-order differences (centred where both neighbours exist in
// the storage grid, one-sided at its edge).  The rest of the source is
// taken to decay as r^-p and is carried outward from the inward neighbour
// q = p - n (n: the outward normal of the point's face, edge or corner):
//   rhs(p) = S(p) + (r_q / r_p)^p (rhs(q) - S(q)).
// Layer k (the points k steps outside the interior box) reads layer k - 1,
// so the layers are separate launches, innermost first.
//
// One thread per (boundary point of the layer, slot): the layer is the
// surface of the box of the interior grown by k, enumerated face by face
// (z faces whole, y faces without their z edges, x faces without either).
// This is a small, memory-bound pass (about 600 bytes per boundary point).
#include <hip/hip_runtime.h>

#include "bssn_internal.h"
#include "bssn_kernels.h"

namespace bssn {
namespace {

// Second-order first derivative of v at storage index j (of N) along the
// axis with element stride st, spacing h.
__device__ __forceinline__ double rad_deriv(const double* v, int64_t idx,
                                            int j, int N, int64_t st,
                                            double h) {
  if (j > 0 && j < N - 1) return (v[idx + st] - v[idx - st]) / (2.0 * h);
  if (j == 0)
    return (-3.0 * v[idx] + 4.0 * v[idx + st] - v[idx + 2 * st]) / (2.0 * h);
  return (3.0 * v[idx] - 4.0 * v[idx - st] + v[idx - 2 * st]) / (2.0 * h);
}

struct RadPoint {
  double S, r;
};

// Wave part of slot s at storage point (i, j, k), and r there.
__device__ __forceinline__ RadPoint rad_wave(const RadiativeArgs& A, int s,
                                             int i, int j, int k) {
  const int g = A.ghost;
  const int N0 = A.n[0] + 2 * g, N1 = A.n[1] + 2 * g, N2 = A.n[2] + 2 * g;
  const double* v = A.u + int64_t(s) * A.sf;
  const int64_t idx = int64_t(k) * A.sz + int64_t(j) * A.sy + i;
  const double x = A.origin[0] + (i - g) * A.h[0];
  const double y = A.origin[1] + (j - g) * A.h[1];
  const double z = A.origin[2] + (k - g) * A.h[2];
  const double r = sqrt(x * x + y * y + z * z);
  const double xd = x * rad_deriv(v, idx, i, N0, 1, A.h[0]) +
                    y * rad_deriv(v, idx, j, N1, A.sy, A.h[1]) +
                    z * rad_deriv(v, idx, k, N2, A.sz, A.h[2]);
  const double v0 = A.v0[s];
  RadPoint p;
  p.S = -v0 * xd / r - v0 * (v[idx] - A.x0[s]) / r;
  p.r = r;
  return p;
}

__global__ void __launch_bounds__(256)
    k_radiative_layer(const RadiativeArgs A, const int layer,
                      const int64_t npts) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (t >= npts) return;
  const int ax = A.n[0] + 2 * layer, ay = A.n[1] + 2 * layer,
            az = A.n[2] + 2 * layer;
  // position on the layer's shell, in [0, a) per axis
  int lx, ly, lz;
  const int64_t fz = int64_t(ax) * ay, fy = int64_t(ax) * (az - 2);
  if (t < 2 * fz) {
    const int64_t m = t % fz;
    lz = t < fz ? 0 : az - 1;
    lx = int(m % ax);
    ly = int(m / ax);
  } else if (t < 2 * fz + 2 * fy) {
    const int64_t u = t - 2 * fz, m = u % fy;
    ly = u < fy ? 0 : ay - 1;
    lx = int(m % ax);
    lz = 1 + int(m / ax);
  } else {
    const int64_t fx = int64_t(ay - 2) * (az - 2);
    const int64_t u = t - 2 * fz - 2 * fy, m = u % fx;
    lx = u < fx ? 0 : ax - 1;
    ly = 1 + int(m % (ay - 2));
    lz = 1 + int(m / (ay - 2));
  }
  const int g = A.ghost;
  const int i = lx - layer + g, j = ly - layer + g, k = lz - layer + g;
  // outward normal and the inward neighbour
  const int sx = i < g ? -1 : (i >= A.n[0] + g ? 1 : 0);
  const int sy = j < g ? -1 : (j >= A.n[1] + g ? 1 : 0);
  const int sz = k < g ? -1 : (k >= A.n[2] + g ? 1 : 0);
  const int qi = i - sx, qj = j - sy, qk = k - sz;
  const RadPoint P = rad_wave(A, s, i, j, k);
  const RadPoint Q = rad_wave(A, s, qi, qj, qk);
  const double ratio = Q.r / P.r;
  double f = 1.0;
  for (int e = 0; e < A.power; ++e) f *= ratio;
  double* out = A.rhs + int64_t(s) * A.sf;
  const double rq = out[int64_t(qk) * A.sz + int64_t(qj) * A.sy + qi];
  out[int64_t(k) * A.sz + int64_t(j) * A.sy + i] = P.S + f * (rq - Q.S);
}

}  // namespace

int64_t radiative_layer_points(const int n[3], int layer) {
  const int64_t ax = n[0] + 2 * layer, ay = n[1] + 2 * layer,
                az = n[2] + 2 * layer;
  return 2 * ax * ay + 2 * ax * (az - 2) + 2 * (ay - 2) * (az - 2);
}

hipError_t launch_radiative(const RadiativeArgs& A, hipStream_t st) {
  for (int layer = 1; layer <= A.ghost; ++layer) {
    const int64_t npts = radiative_layer_points(A.n, layer);
    const int64_t nb = (npts + 255) / 256;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_radiative_layer, dim3(unsigned(nb), NSLOT),
                       dim3(256), 0, st, A, layer, npts);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace bssn
