// bssn_amr.hip -- the mesh-refinement glue kernels (Einstein Toolkit paper,
// the Carpet mesh-refinement part of the framework section: Berger-Oliger
// time stepping, fine-grid boundaries by interpolation in space and time,
// the fine solution put back into the coarse grid).
//
// Both kernels walk an op list built on the host (bssn_amr_plan.cpp), one
// thread per (op, slot):
//   k_amr_fill      a ghost point of a refined patch: a copy from a sibling
//                   patch's interior, or the tricubic interpolation of the
//                   coarse patch (per-axis weights (-7, 105, 35, -5)/128 or
//                   their mirror, the fine point a quarter coarse spacing
//                   from a coarse point) combined over up to three coarse
//                   time levels with Lagrange weights in time;
//   k_amr_restrict  a coarse interior point covered by a refined patch: the
//                   tricubic midpoint interpolation (-1, 9, 9, -1)/16 of
//                   the fine storage around it.
// Memory-bound: a copy moves 16 B per slot; an interpolation reads 64
// points, most of them shared with its neighbours through the caches.
#include <hip/hip_runtime.h>

#include "bssn_internal.h"
#include "bssn_kernels.h"

namespace bssn {
namespace {

__device__ __forceinline__ double w_quarter(int phase, int m) {
  // phase 0: the point at 1.25 of the block's nodes 0..3; phase 1: at 1.75
  const int k = phase ? 3 - m : m;
  return k == 0 ? -7.0 / 128.0
         : k == 1 ? 105.0 / 128.0
         : k == 2 ? 35.0 / 128.0
                  : -5.0 / 128.0;
}

__device__ __forceinline__ double w_mid(int m) {
  return (m == 0 || m == 3) ? -1.0 / 16.0 : 9.0 / 16.0;
}

// Workgroups are dealt to the 8 XCDs in turn (linear id mod 8).  Give each
// XCD a contiguous eighth of the (slot, chunk of 256 ops) space instead, so
// that neighbouring ops -- which read overlapping coarse blocks -- share an
// L2.  nwg is the launch's workgroup count, a multiple of 8.
struct Work {
  int64_t t;  // op index
  int s;      // slot
  bool live;
};
__device__ __forceinline__ Work xcd_work(int64_t nops, int64_t nchunks) {
  const int64_t nwg = gridDim.x, b = blockIdx.x;
  const int64_t id = (b % 8) * (nwg / 8) + b / 8;
  Work w;
  w.s = int(id / nchunks);
  w.t = (id % nchunks) * 256 + threadIdx.x;
  w.live = id < nchunks * NSLOT && w.t < nops;
  return w;
}

__global__ void __launch_bounds__(256)
    k_amr_fill(const AmrOp* __restrict__ ops, const int64_t nops,
               const int64_t nchunks, const AmrGeo* __restrict__ geo,
               double* const* __restrict__ u, const AmrTime T) {
  const Work w = xcd_work(nops, nchunks);
  if (!w.live) return;
  const int64_t t = w.t;
  const int s = w.s;
  const AmrOp op = ops[t];
  const AmrGeo gd = geo[op.dpatch], gs = geo[op.spatch];
  double* d = u[op.dpatch] + int64_t(s) * gd.sf + op.dst;
  if (!(op.code & AMR_PROLONG)) {
    *d = u[op.spatch][int64_t(s) * gs.sf + op.src];
    return;
  }
  const int px = (op.code >> 1) & 1, py = (op.code >> 2) & 1,
            pz = (op.code >> 3) & 1;
  double val = 0.0;
  for (int l = 0; l < T.ntl; ++l) {
    const double* c = T.tab[l][op.spatch] + int64_t(s) * gs.sf + op.src;
    double acc = 0.0;
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          acc += w_quarter(pz, k) * w_quarter(py, j) * w_quarter(px, i) *
                 c[k * gs.sz + j * gs.sy + i];
    val += T.w[l] * acc;
  }
  *d = val;
}

__global__ void __launch_bounds__(256)
    k_amr_restrict(const AmrOp* __restrict__ ops, const int64_t nops,
                   const int64_t nchunks, const AmrGeo* __restrict__ geo,
                   double* const* __restrict__ coarse,
                   const double* const* __restrict__ fine) {
  const Work w = xcd_work(nops, nchunks);
  if (!w.live) return;
  const int64_t t = w.t;
  const int s = w.s;
  const AmrOp op = ops[t];
  const AmrGeo gd = geo[op.dpatch], gs = geo[op.spatch];
  const double* c = fine[op.spatch] + int64_t(s) * gs.sf + op.src;
  double acc = 0.0;
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        acc += w_mid(k) * w_mid(j) * w_mid(i) * c[k * gs.sz + j * gs.sy + i];
  coarse[op.dpatch][int64_t(s) * gd.sf + op.dst] = acc;
}

}  // namespace

hipError_t launch_amr_fill(const AmrOp* ops, int64_t nops, const AmrGeo* geo,
                           double* const* u, const AmrTime& T,
                           hipStream_t st) {
  if (nops <= 0) return hipSuccess;
  const int64_t nchunks = (nops + 255) / 256;
  const int64_t nwg = (nchunks * NSLOT + 7) / 8 * 8;
  if (nwg > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_amr_fill, dim3(unsigned(nwg)), dim3(256), 0, st, ops,
                     nops, nchunks, geo, u, T);
  return hipGetLastError();
}

hipError_t launch_amr_restrict(const AmrOp* ops, int64_t nops,
                               const AmrGeo* geo, double* const* coarse,
                               const double* const* fine, hipStream_t st) {
  if (nops <= 0) return hipSuccess;
  const int64_t nchunks = (nops + 255) / 256;
  const int64_t nwg = (nchunks * NSLOT + 7) / 8 * 8;
  if (nwg > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_amr_restrict, dim3(unsigned(nwg)), dim3(256), 0, st,
                     ops, nops, nchunks, geo, coarse, fine);
  return hipGetLastError();
}

}  // namespace bssn
