// bssn_amr.hip -- the mesh-refinement glue kernels (Einstein Toolkit paper,
// the Carpet mesh-refinement part of the framework section: Berger-Oliger
// time stepping, fine-grid boundaries by interpolation in space and time,
// the fine solution put back into the coarse grid).
//
// Lists built on the host (bssn_amr_plan.cpp):
//   k_amr_fill      one thread per op, all slots: a ghost point copied
//                   from a sibling patch's interior;
//   k_amr_prolong   one workgroup per (tile, slot): the prolonged ghost
//                   points of an 8 x 8 x 8 box of a refined patch, the
//                   tricubic interpolation of the coarse patch (per-axis
//                   weights (-7, 105, 35, -5)/128 or their mirror, the fine
//                   point a quarter coarse spacing from a coarse point)
//                   combined over up to three coarse time levels with
//                   Lagrange weights in time, from the coarse region staged
//                   in LDS;
//   k_amr_restrict  one thread per (op, group of slots): a coarse
//                   interior point covered by a refined patch: the
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
// XCD a contiguous eighth of the (slot group, chunk of 256 ops) space
// instead, so that neighbouring ops -- which read overlapping fine blocks
// -- share an L2.  nwg is the launch's workgroup count, a multiple of 8.
struct Work {
  int64_t t;  // op index
  int g;      // slot group
  bool live;
};
__device__ __forceinline__ Work xcd_work(int64_t nops, int64_t nchunks,
                                         int ngroups) {
  const int64_t nwg = gridDim.x, b = blockIdx.x;
  const int64_t id = (b % 8) * (nwg / 8) + b / 8;
  Work w;
  w.g = int(id / nchunks);
  w.t = (id % nchunks) * 256 + threadIdx.x;
  w.live = id < nchunks * ngroups && w.t < nops;
  return w;
}

// Slots per restriction thread: the op is read once per group (with one
// slot per thread the op list, larger than an L2, was read from HBM for
// every slot).
constexpr int RESTRICT_SLOTS = 5;
static_assert(NSLOT % RESTRICT_SLOTS == 0, "slots per thread");

// One thread per copy op, all 25 slots: the op is read once (a thread per
// (op, slot) read it 25 times, from HBM, as the list outgrows the L2), the
// slots' loads are all in flight before the first store.  A copy's source
// (a sibling's interior) and destination (a ghost point) never overlap.
__global__ void __launch_bounds__(256)
    k_amr_fill(const AmrOp* __restrict__ ops, const int64_t nops,
               const AmrGeo* __restrict__ geo, double* const* __restrict__ u) {
  const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (t >= nops) return;
  const AmrOp op = ops[t];
  const int64_t sfd = geo[op.dpatch].sf, sfs = geo[op.spatch].sf;
  const double* src = u[op.spatch] + op.src;
  double* dst = u[op.dpatch] + op.dst;
  double v[NSLOT];
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) v[s] = src[s * sfs];
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) dst[s * sfd] = v[s];
}

__global__ void __launch_bounds__(256)
    k_amr_restrict(const AmrOp* __restrict__ ops, const int64_t nops,
                   const int64_t nchunks, const AmrGeo* __restrict__ geo,
                   double* const* __restrict__ coarse,
                   const double* const* __restrict__ fine) {
  const Work w = xcd_work(nops, nchunks, NSLOT / RESTRICT_SLOTS);
  if (!w.live) return;
  const AmrOp op = ops[w.t];
  const AmrGeo gd = geo[op.dpatch], gs = geo[op.spatch];
  const int s0 = w.g * RESTRICT_SLOTS;
  const double* c0 = fine[op.spatch] + int64_t(s0) * gs.sf + op.src;
  double* d0 = coarse[op.dpatch] + int64_t(s0) * gd.sf + op.dst;
#pragma unroll 1
  for (int q = 0; q < RESTRICT_SLOTS; ++q) {
    const double* c = c0 + int64_t(q) * gs.sf;
    double acc = 0.0;
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          acc += w_mid(k) * w_mid(j) * w_mid(i) * c[k * gs.sz + j * gs.sy + i];
    d0[int64_t(q) * gd.sf] = acc;
  }
}

// One workgroup per (tile, slot): stage the tile's coarse region in LDS
// with the time levels combined (Lagrange weights in time, the same for
// every point), then apply the tensor-product weights one axis at a time
// over the bounding box of the tile's filled points, each pass from LDS to
// LDS: x (every region row, the box's x points), y, then z at the filled
// points only.  Each point's sum is the same sequence of multiply-adds as
// the point-wise form (x innermost, then y, then z), with 12 LDS reads per
// point instead of 64.
__global__ void __launch_bounds__(256)
    k_amr_prolong(const AmrTile* __restrict__ tiles, const int64_t ntiles,
                  const AmrGeo* __restrict__ geo,
                  double* const* __restrict__ u, const AmrTime T) {
  // the region (pitches 9 and 81 spread a wave's reads over the LDS banks),
  // then the x sums [region z][region y][box x] and the y sums
  // [region z][box y][box x], both with pitches 9 and 72
  __shared__ double reg[8 * 81];
  __shared__ double xs[8 * 72];
  __shared__ double ys[8 * 72];
  const int64_t nwg = gridDim.x, b = blockIdx.x;
  const int64_t id = (b % 8) * (nwg / 8) + b / 8;
  if (id >= ntiles * NSLOT) return;  // uniform over the workgroup
  const int s = int(id / ntiles);
  // fields read from the tile in memory: a local copy of the struct, indexed
  // at run time (mask words), would live in scratch
  const AmrTile* tp = tiles + id % ntiles;
  const int dpatch = tp->dpatch, spatch = tp->spatch;
  const AmrGeo gs = geo[spatch], gd = geo[dpatch];
  const int cx = tp->c[0], cy = tp->c[1], cz = tp->c[2];
  const int nreg = cx * cy * cz;
  const int64_t src0 = tp->src0 + int64_t(s) * gs.sf;
  // every load of the region issued before the first LDS store (a region
  // holds at most 512 values: two per thread per time level), so their
  // latencies overlap
  double v[3][2];
  int lds_at[2];
  bool have[2];
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const int e = threadIdx.x + it * 256;
    have[it] = e < nreg;
    const int x = e % cx, r = e / cx, y = r % cy, z = r / cy;
    lds_at[it] = z * 81 + y * 9 + x;
    const int64_t off = int64_t(z) * gs.sz + int64_t(y) * gs.sy + x;
#pragma unroll
    for (int l = 0; l < 3; ++l)
      if (have[it] && l < T.ntl) v[l][it] = T.tab[l][spatch][src0 + off];
  }
#pragma unroll
  for (int it = 0; it < 2; ++it)
    if (have[it]) {
      double t = T.w[0] * v[0][it];
      if (T.ntl > 1) t += T.w[1] * v[1][it];
      if (T.ntl > 2) t += T.w[2] * v[2][it];
      reg[lds_at[it]] = t;
    }
  const int code = tp->code;
  const int ex = code & 1, ey = (code >> 1) & 1, ez = (code >> 2) & 1;
  const int r0x = tp->r0[0], r0y = tp->r0[1], r0z = tp->r0[2];
  const int lx = tp->lo[0], ly = tp->lo[1], lz = tp->lo[2];
  const int mx = tp->m[0], my = tp->m[1], mz = tp->m[2];
  __syncthreads();
  // x pass: entry (i, y, z) of an 8 x 8 x 8 index space, box x = lx + i
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const int e = threadIdx.x + it * 256;
    const int i = e & 7, y = (e >> 3) & 7, z = e >> 6;
    if (i < mx && y < cy && z < cz) {
      const int fx = lx + i;
      const int bx = r0x + (ex + fx) / 2, px = (ex + fx) & 1;
      const double* c = reg + z * 81 + y * 9 + bx;
      double xsum = 0.0;
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) xsum += w_quarter(px, ii) * c[ii];
      xs[z * 72 + y * 9 + i] = xsum;
    }
  }
  __syncthreads();
  // y pass: entry (i, j, z), box y = ly + j
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const int e = threadIdx.x + it * 256;
    const int i = e & 7, j = (e >> 3) & 7, z = e >> 6;
    if (i < mx && j < my && z < cz) {
      const int fy = ly + j;
      const int by = r0y + (ey + fy) / 2, py = (ey + fy) & 1;
      const double* c = xs + z * 72 + by * 9 + i;
      double ysum = 0.0;
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) ysum += w_quarter(py, jj) * c[jj * 9];
      ys[z * 72 + j * 9 + i] = ysum;
    }
  }
  __syncthreads();
  // z pass at the filled points: entry (i, j, k), box z = lz + k
  double* dst = u[dpatch] + int64_t(s) * gd.sf + tp->dst0;
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const int e = threadIdx.x + it * 256;
    const int i = e & 7, j = (e >> 3) & 7, k = e >> 6;
    const int fx = lx + i, fy = ly + j, fz = lz + k;
    const int pt = fx + 8 * fy + 64 * fz;
    if (i < mx && j < my && k < mz &&
        ((tp->mask[pt >> 6] >> (pt & 63)) & 1)) {
      const int bz = r0z + (ez + fz) / 2, pz = (ez + fz) & 1;
      const double* c = ys + bz * 72 + j * 9 + i;
      double zsum = 0.0;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) zsum += w_quarter(pz, kk) * c[kk * 72];
      dst[fz * gd.sz + fy * gd.sy + fx] = zsum;
    }
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
  const int64_t nwg = (nops + 255) / 256;
  if (nwg > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_amr_fill, dim3(unsigned(nwg)), dim3(256), 0, st, ops,
                     nops, geo, u);
  return hipGetLastError();
}

hipError_t launch_amr_restrict(const AmrOp* ops, int64_t nops,
                               const AmrGeo* geo, double* const* coarse,
                               const double* const* fine, hipStream_t st) {
  if (nops <= 0) return hipSuccess;
  const int64_t nchunks = (nops + 255) / 256;
  const int64_t nwg = (nchunks * (NSLOT / RESTRICT_SLOTS) + 7) / 8 * 8;
  if (nwg > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_amr_restrict, dim3(unsigned(nwg)), dim3(256), 0, st,
                     ops, nops, nchunks, geo, coarse, fine);
  return hipGetLastError();
}

}  // namespace bssn
