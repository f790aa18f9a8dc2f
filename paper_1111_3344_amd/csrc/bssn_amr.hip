// bssn_amr.hip -- the mesh-refinement glue kernels (Einstein Toolkit paper,
// the Carpet mesh-refinement part of the framework section: Berger-Oliger
// time stepping, fine-grid boundaries by interpolation in space and time,
// the fine solution put back into the coarse grid).
//
// Lists built on the host (bssn_amr_plan.cpp):
//   k_amr_fill      one thread per (op, slot): a ghost point copied from a
//                   sibling patch's interior;
//   k_amr_prolong   one workgroup per (tile, slot): the prolonged ghost
//                   points of an 8 x 8 x 8 box of a refined patch, the
//                   tricubic interpolation of the coarse patch (per-axis
//                   weights (-7, 105, 35, -5)/128 or their mirror, the fine
//                   point a quarter coarse spacing from a coarse point)
//                   combined over up to three coarse time levels with
//                   Lagrange weights in time, from the coarse region staged
//                   in LDS;
//   k_amr_restrict  one thread per (op, slot): a coarse interior point
//                   covered by a refined patch: the
//                   tricubic midpoint interpolation (-1, 9, 9, -1)/16 of
//                   the fine storage around it.
// Memory-bound: a copy moves 16 B per slot; a tile reads its coarse region
// once per time level and writes its points.
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
               double* const* __restrict__ u) {
  const Work w = xcd_work(nops, nchunks);
  if (!w.live) return;
  const AmrOp op = ops[w.t];
  const AmrGeo gd = geo[op.dpatch], gs = geo[op.spatch];
  u[op.dpatch][int64_t(w.s) * gd.sf + op.dst] =
      u[op.spatch][int64_t(w.s) * gs.sf + op.src];
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

// One workgroup per (tile, slot): stage the tile's coarse region for every
// time level in LDS (coalesced rows), then each masked fine point of the
// box interpolates from LDS with the same weights and order as k_amr_fill.
__global__ void __launch_bounds__(256)
    k_amr_prolong(const AmrTile* __restrict__ tiles, const int64_t ntiles,
                  const AmrGeo* __restrict__ geo,
                  double* const* __restrict__ u, const AmrTime T) {
  __shared__ double reg[3 * 512];
  const int64_t nwg = gridDim.x, b = blockIdx.x;
  const int64_t id = (b % 8) * (nwg / 8) + b / 8;
  if (id >= ntiles * NSLOT) return;  // uniform over the workgroup
  const int s = int(id / ntiles);
  const AmrTile tl = tiles[id % ntiles];
  const AmrGeo gs = geo[tl.spatch], gd = geo[tl.dpatch];
  const int cx = tl.c[0], cy = tl.c[1], cz = tl.c[2];
  const int nreg = cx * cy * cz;
  for (int l = 0; l < T.ntl; ++l) {
    const double* src = T.tab[l][tl.spatch] + int64_t(s) * gs.sf + tl.src0;
    for (int e = threadIdx.x; e < nreg; e += 256) {
      const int x = e % cx, r = e / cx, y = r % cy, z = r / cy;
      reg[l * 512 + z * 64 + y * 8 + x] = src[z * gs.sz + y * gs.sy + x];
    }
  }
  __syncthreads();
  double* dst = u[tl.dpatch] + int64_t(s) * gd.sf + tl.dst0;
  const int ex = tl.code & 1, ey = (tl.code >> 1) & 1, ez = (tl.code >> 2) & 1;
  for (int pt = threadIdx.x; pt < 512; pt += 256) {
    if (!((tl.mask[pt >> 6] >> (pt & 63)) & 1)) continue;
    const int i = pt & 7, j = (pt >> 3) & 7, k = pt >> 6;
    const int bx = tl.r0[0] + (ex + i) / 2, by = tl.r0[1] + (ey + j) / 2,
              bz = tl.r0[2] + (ez + k) / 2;
    const int px = (ex + i) & 1, py = (ey + j) & 1, pz = (ez + k) & 1;
    const int base = bz * 64 + by * 8 + bx;
    double val = 0.0;
    for (int l = 0; l < T.ntl; ++l) {
      const double* c = reg + l * 512 + base;
      double acc = 0.0;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
#pragma unroll
          for (int ii = 0; ii < 4; ++ii)
            acc += w_quarter(pz, kk) * w_quarter(py, jj) * w_quarter(px, ii) *
                   c[kk * 64 + jj * 8 + ii];
      val += T.w[l] * acc;
    }
    dst[k * gd.sz + j * gd.sy + i] = val;
  }
}

}  // namespace

hipError_t launch_amr_prolong(const AmrTile* tiles, int64_t ntiles,
                              const AmrGeo* geo, double* const* u,
                              const AmrTime& T, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  const int64_t nwg = (ntiles * NSLOT + 7) / 8 * 8;
  if (nwg > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_amr_prolong, dim3(unsigned(nwg)), dim3(256), 0, st,
                     tiles, ntiles, geo, u, T);
  return hipGetLastError();
}

hipError_t launch_amr_fill(const AmrOp* ops, int64_t nops, const AmrGeo* geo,
                           double* const* u, hipStream_t st) {
  if (nops <= 0) return hipSuccess;
  const int64_t nchunks = (nops + 255) / 256;
  const int64_t nwg = (nchunks * NSLOT + 7) / 8 * 8;
  if (nwg > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_amr_fill, dim3(unsigned(nwg)), dim3(256), 0, st, ops,
                     nops, nchunks, geo, u);
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
