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
// Layer k (the points k steps outside the interior box) is defined from
// layer k - 1; the recursion telescopes to the interior (k_radiative), so
// one launch computes every layer.  This is a small, memory-bound pass
// (about 600 bytes per boundary point).
#include <hip/hip_runtime.h>

#include "bssn_internal.h"
#include "bssn_kernels.h"

namespace bssn {
namespace {

// Second-order first derivative of v at storage index j (of N) along the
// axis with element stride st; i2h = 1 / (2 h).
__device__ __forceinline__ double rad_deriv(const double* v, int64_t idx,
                                            int j, int N, int64_t st,
                                            double i2h) {
  if (j > 0 && j < N - 1) return (v[idx + st] - v[idx - st]) * i2h;
  if (j == 0)
    return (-3.0 * v[idx] + 4.0 * v[idx + st] - v[idx + 2 * st]) * i2h;
  return (3.0 * v[idx] - 4.0 * v[idx - st] + v[idx - 2 * st]) * i2h;
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
  const double xd = x * rad_deriv(v, idx, i, N0, 1, A.i2h[0]) +
                    y * rad_deriv(v, idx, j, N1, A.sy, A.i2h[1]) +
                    z * rad_deriv(v, idx, k, N2, A.sz, A.i2h[2]);
  RadPoint p;
  p.S = -A.v0[s] * (xd + (v[idx] - A.x0[s])) / r;
  p.r = r;
  return p;
}

// Storage point (i, j, k) of boundary point t (32-bit counts, checked on the
// host), numbered as described below; false past the last one.
__device__ __forceinline__ bool boundary_point(const RadiativeArgs& A,
                                               uint32_t t, uint32_t na,
                                               uint32_t nb, uint32_t nc,
                                               int& i, int& j, int& k) {
  const int g = A.ghost;
  const uint32_t N0 = A.n[0] + 2 * g, N1 = A.n[1] + 2 * g;
  if (t < na) {
    const uint32_t plane = t / (N0 * N1), m = t - plane * (N0 * N1);
    k = int(plane) < g ? int(plane) : int(plane) - g + A.n[2] + g;
    j = int(m / N0);
    i = int(m - uint32_t(j) * N0);
  } else if (t < na + nb) {
    const uint32_t u = t - na, row = u / N0;
    i = int(u - row * N0);
    const uint32_t rk = row / uint32_t(2 * g);
    const int jr = int(row - rk * uint32_t(2 * g));
    k = g + int(rk);
    j = jr < g ? jr : jr - g + A.n[1] + g;
  } else if (t < na + nb + nc) {
    const uint32_t u = t - na - nb;
    const uint32_t row = u / uint32_t(2 * g);
    const int e = int(u - row * uint32_t(2 * g));
    const uint32_t kk = row / uint32_t(A.n[1]);
    j = g + int(row - kk * uint32_t(A.n[1]));
    k = g + int(kk);
    i = e < g ? e : e - g + A.n[0] + g;
  } else {
    return false;
  }
  return true;
}

// One thread per (boundary point, slot).  The boundary points (all ghost
// layers) are numbered in three parts, x fastest where rows are whole:
//   A  the z slabs (k < g or k >= n2 + g): whole planes;
//   B  in interior planes, the y slabs: whole rows;
//   C  in interior rows, the g points at each x end.
// The layer recursion telescopes: following q = p - n from p reaches, after
// as many steps as p's layer, the interior point `root` (p clamped into the
// interior box per axis), and the factors multiply to (r_root / r_p)^power:
//   rhs(p) = S(p) + (r_root / r_p)^power (rhs(root) - S(root)).
__global__ void __launch_bounds__(256)
    k_radiative(const RadiativeArgs A, const uint32_t na, const uint32_t nb,
                const uint32_t nc) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  const int g = A.ghost;
  int i, j, k;
  if (!boundary_point(A, t, na, nb, nc, i, j, k)) return;
  const int ri = i < g ? g : (i >= A.n[0] + g ? A.n[0] + g - 1 : i);
  const int rj = j < g ? g : (j >= A.n[1] + g ? A.n[1] + g - 1 : j);
  const int rk = k < g ? g : (k >= A.n[2] + g ? A.n[2] + g - 1 : k);
  const RadPoint P = rad_wave(A, s, i, j, k);
  const RadPoint Q = rad_wave(A, s, ri, rj, rk);
  const double ratio = Q.r / P.r;
  double f = 1.0;
  for (int e = 0; e < A.power; ++e) f *= ratio;
  double* out = A.rhs + int64_t(s) * A.sf;
  const double rr = out[int64_t(rk) * A.sz + int64_t(rj) * A.sy + ri];
  out[int64_t(k) * A.sz + int64_t(j) * A.sy + i] = P.S + f * (rr - Q.S);
}

// The same boundary points and right-hand side, each fed into the RK4
// stage update of its point (stage s, step dt; the arithmetic of the fused
// interior stage):
//   s = 0: acc = u_n + dt/6 k,  out = u_n + dt/2 k
//   s = 1: acc = acc + dt/3 k,  out = u_n + dt/2 k
//   s = 2: acc = acc + dt/3 k,  out = u_n + dt k
//   s = 3:                      out = acc + dt/6 k
__global__ void __launch_bounds__(256)
    k_radiative_stage(const RadiativeArgs A, const RadStage S,
                      const uint32_t na, const uint32_t nb,
                      const uint32_t nc) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  const int g = A.ghost;
  int i, j, k;
  if (!boundary_point(A, t, na, nb, nc, i, j, k)) return;
  const int ri = i < g ? g : (i >= A.n[0] + g ? A.n[0] + g - 1 : i);
  const int rj = j < g ? g : (j >= A.n[1] + g ? A.n[1] + g - 1 : j);
  const int rk = k < g ? g : (k >= A.n[2] + g ? A.n[2] + g - 1 : k);
  const RadPoint P = rad_wave(A, s, i, j, k);
  const RadPoint Q = rad_wave(A, s, ri, rj, rk);
  const double ratio = Q.r / P.r;
  double f = 1.0;
  for (int e = 0; e < A.power; ++e) f *= ratio;
  const int64_t so = int64_t(s) * A.sf;
  const double rr = A.rhs[so + int64_t(rk) * A.sz + int64_t(rj) * A.sy + ri];
  const double kv = P.S + f * (rr - Q.S);
  const int64_t o = so + int64_t(k) * A.sz + int64_t(j) * A.sy + i;
  const double dt = S.dt;
  if (S.stage == ST_0) {
    const double un = S.u_n[o];
    S.acc[o] = un + (dt / 6.0) * kv;
    S.out[o] = un + (dt / 2.0) * kv;
  } else if (S.stage == ST_3) {
    S.out[o] = S.acc[o] + (dt / 6.0) * kv;
  } else {
    const double c = S.stage == ST_1 ? dt / 2.0 : dt;
    const double un = S.u_n[o], ac = S.acc[o];
    S.acc[o] = ac + (dt / 3.0) * kv;
    S.out[o] = un + c * kv;
  }
}

}  // namespace

hipError_t launch_radiative_stage(const RadiativeArgs& A, const RadStage& S,
                                  hipStream_t st) {
  const int64_t g = A.ghost;
  const int64_t N0 = A.n[0] + 2 * g, N1 = A.n[1] + 2 * g;
  const int64_t na = 2 * g * N1 * N0;
  const int64_t nb = int64_t(A.n[2]) * 2 * g * N0;
  const int64_t nc = int64_t(A.n[2]) * A.n[1] * 2 * g;
  // boundary points are counted in 32 bits
  if (na + nb + nc + 255 > 0xffffffffll) return hipErrorInvalidValue;
  const int64_t blocks = (na + nb + nc + 255) / 256;
  hipLaunchKernelGGL(k_radiative_stage, dim3(unsigned(blocks), NSLOT),
                     dim3(256), 0, st, A, S, uint32_t(na), uint32_t(nb),
                     uint32_t(nc));
  return hipGetLastError();
}

hipError_t launch_radiative(const RadiativeArgs& A, hipStream_t st) {
  const int64_t g = A.ghost;
  const int64_t N0 = A.n[0] + 2 * g, N1 = A.n[1] + 2 * g;
  const int64_t na = 2 * g * N1 * N0;
  const int64_t nb = int64_t(A.n[2]) * 2 * g * N0;
  const int64_t nc = int64_t(A.n[2]) * A.n[1] * 2 * g;
  // boundary points are counted in 32 bits
  if (na + nb + nc + 255 > 0xffffffffll) return hipErrorInvalidValue;
  const int64_t blocks = (na + nb + nc + 255) / 256;
  hipLaunchKernelGGL(k_radiative, dim3(unsigned(blocks), NSLOT), dim3(256), 0,
                     st, A, uint32_t(na), uint32_t(nb), uint32_t(nc));
  return hipGetLastError();
}

}  // namespace bssn
