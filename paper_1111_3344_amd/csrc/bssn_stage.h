// bssn_stage.h -- fused BSSN right-hand side + classical RK4 stage kernels.
//
// One thread per interior point; a workgroup covers a BX x BY tile of one
// z-plane.  Stencil values are read straight from HBM through the vector L1
// and L2 caches with raw buffer loads: each slot gets a buffer resource based
// at the slot start, the lane's offset is the byte offset of the stencil's
// lowest corner (x-R, y-R, z-R) and every tap adds a non-negative
// compile-time multiple of the row/plane pitch in the scalar offset, so no
// per-tap vector address arithmetic is issued.  Offsets beyond the buffer
// read as zero instead of faulting.  Periodic grids wrap the indices per lane
// (small grids only).
//
// The RK4 epilogue is fused: the stage's k never goes to memory.
#pragma once
#include <hip/hip_runtime.h>

#include "bssn_internal.h"
#include "bssn_point.h"

namespace bssn {

constexpr int32_t kRsrcWord3 = 0x00020000;  // gfx9 raw 32-bit buffer

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const double* base,
                                                       int32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, bytes,
                                           kRsrcWord3);
}

// Buffer resource of slot s built where it is used: the base and the slot
// stride go through an opaque scalar move, so neither the per-slot
// descriptors nor the per-slot offsets s*sf of a loop body are hoisted out
// of the loop (25 slots x 3 buffers x 4 SGPRs, or 25 x 2 SGPRs, would be
// spilled to VGPR lanes and moved back on every use).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t slot_rsrc(const double* u,
                                                            int64_t sf, int s,
                                                            int32_t nbytes) {
  const double* b = u;
  int64_t o = sf;
  asm volatile("" : "+s"(b), "+s"(o));
  return rsrc(b + s * o, nbytes);
}

__device__ __forceinline__ double bload(__amdgpu_buffer_rsrc_t r,
                                        uint32_t voff, uint32_t soff) {
  auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0);
  return __builtin_bit_cast(double, v);
}

__device__ __forceinline__ double bload_nt(__amdgpu_buffer_rsrc_t r,
                                        uint32_t voff) {
  auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, 0, 2);
  return __builtin_bit_cast(double, v);
}
__device__ __forceinline__ void bstore_nt(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                       double x) {
  __builtin_amdgcn_raw_buffer_store_b64(
      __builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(
                             r, 0, 0, 0)),
                         x),
      r, (int)voff, 0, 2);
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                       double x) {
  __builtin_amdgcn_raw_buffer_store_b64(
      __builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(
                             r, 0, 0, 0)),
                         x),
      r, (int)voff, 0, 0);
}

// Static boundary: offsets relative to the stencil's lowest corner.
template <int R>
struct LdStatic {
  const double* u;
  int64_t sf;
  int32_t nbytes;     // bytes of one slot (buffer range)
  uint32_t vlo;       // byte offset of (x-R, y-R, z-R) within a slot
  uint32_t str[3];    // bytes per step along x, y, z
  __device__ __forceinline__ double at(int s, uint32_t soff) const {
    return bload(rsrc(u + s * sf, nbytes), vlo, soff);
  }
  __device__ __forceinline__ void enter(int) const { BSSN_PHASE(); }
  __device__ __forceinline__ double g(int s) const { return c(s); }
  __device__ __forceinline__ double c(int s) const {
    return at(s, R * (str[0] + str[1] + str[2]));
  }
  __device__ __forceinline__ double ax(int s, int a, int k) const {
    return at(s, R * (str[0] + str[1] + str[2]) + k * (int)str[a]);
  }
  __device__ __forceinline__ double pl(int s, int a, int i, int b,
                                       int j) const {
    return at(s, R * (str[0] + str[1] + str[2]) + i * (int)str[a] +
                     j * (int)str[b]);
  }
};

// Periodic boundary: per-lane wrapped offsets for every reach.
template <int R>
struct LdPeriodic {
  const double* u;
  int64_t sf;
  int32_t nbytes;
  uint32_t o[3][2 * R + 1];  // byte offset contribution of axis a at k
  __device__ __forceinline__ double at(int s, uint32_t v) const {
    return bload(rsrc(u + s * sf, nbytes), v, 0);
  }
  __device__ __forceinline__ void enter(int) const { BSSN_PHASE(); }
  __device__ __forceinline__ double g(int s) const { return c(s); }
  __device__ __forceinline__ double c(int s) const {
    return at(s, o[0][R] + o[1][R] + o[2][R]);
  }
  __device__ __forceinline__ double ax(int s, int a, int k) const {
    uint32_t v = o[0][R] + o[1][R] + o[2][R];
    v += o[a][R + k] - o[a][R];
    return at(s, v);
  }
  __device__ __forceinline__ double pl(int s, int a, int i, int b,
                                       int j) const {
    const int cidx = 3 - a - b;
    return at(s, o[a][R + i] + o[b][R + j] + o[cidx][R]);
  }
};

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}

// Minimum lapse over the workgroup's points: the mixed-precision routing
// predicate, identical in the FP32 and the FP64 kernel of a pair.
__device__ __forceinline__ bool tile_needs_fp64(const Patch& P, bool active,
                                                uint32_t vc, int32_t nbytes,
                                                double thr) {
  __shared__ double wmin[16];
  double a = 1.0e300;
  if (active) a = bload(rsrc(P.u_s + ALP * P.sf, nbytes), vc, 0);
  a = wave_min(a);
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  const int nw = (blockDim.x * blockDim.y + 63) >> 6;
  if ((tid & 63) == 0) wmin[tid >> 6] = a;
  __syncthreads();
  double m = wmin[0];
  for (int w = 1; w < nw; ++w) m = fmin(m, wmin[w]);
  // every wave has read wmin before any wave can overwrite it for the
  // next plane of a multi-plane workgroup
  __syncthreads();
  return m < thr;
}

// Stage epilogue: k -> acc / out (FP64), in two halves so a caller can
// issue the loads early.  epilogue_load reads u_n (stages 0..2) and acc
// (stages 1..3) at byte offset vc of every slot; epilogue_store writes acc
// and the stage output.  Every load is issued before the first store (the
// compiler cannot prove the stores of one slot miss the loads of the next,
// so interleaving them would serialise 25 round trips).
__device__ __forceinline__ void epilogue_load(const Patch& P, int stage,
                                              uint32_t vc, int32_t nbytes,
                                              double (&un)[NSLOT],
                                              double (&ac)[NSLOT]) {
  if (stage != ST_3 && stage != ST_RHS) {
#pragma unroll
    for (int s = 0; s < NSLOT; ++s)
      un[s] = bload_nt(slot_rsrc(P.u_n, P.sf, s, nbytes), vc);
  }
  if (stage != ST_0 && stage != ST_RHS) {
#pragma unroll
    for (int s = 0; s < NSLOT; ++s)
      ac[s] = bload_nt(slot_rsrc(P.acc, P.sf, s, nbytes), vc);
  }
}
// Memory instructions of the two halves for one wave.
__device__ __forceinline__ int epilogue_loads(int stage) {
  return stage == ST_RHS ? 0
         : (stage == ST_0 || stage == ST_3) ? NSLOT
                                             : 2 * NSLOT;
}
__device__ __forceinline__ int epilogue_stores(int stage) {
  return (stage == ST_RHS || stage == ST_3) ? NSLOT : 2 * NSLOT;
}

template <typename T>
__device__ __forceinline__ void epilogue_store(const Patch& P, int stage,
                                               const T (&r)[NSLOT],
                                               uint32_t vc, int32_t nbytes,
                                               const double (&un)[NSLOT],
                                               const double (&ac)[NSLOT]) {
  const double dt = P.dt;
  if (stage == ST_RHS) {
#pragma unroll
    for (int s = 0; s < NSLOT; ++s)
      bstore_nt(slot_rsrc(P.out, P.sf, s, nbytes), vc, double(r[s]));
  } else if (stage == ST_3) {
#pragma unroll
    for (int s = 0; s < NSLOT; ++s)
      bstore_nt(slot_rsrc(P.out, P.sf, s, nbytes), vc,
                ac[s] + (dt / 6.0) * double(r[s]));
  } else if (stage == ST_0) {
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) {
      const double k = double(r[s]);
      bstore_nt(slot_rsrc(P.acc, P.sf, s, nbytes), vc,
                un[s] + (dt / 6.0) * k);
      bstore_nt(slot_rsrc(P.out, P.sf, s, nbytes), vc,
                un[s] + (dt / 2.0) * k);
    }
  } else {
    const double c = stage == ST_1 ? dt / 2.0 : dt;
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) {
      const double k = double(r[s]);
      bstore_nt(slot_rsrc(P.acc, P.sf, s, nbytes), vc,
                ac[s] + (dt / 3.0) * k);
      bstore_nt(slot_rsrc(P.out, P.sf, s, nbytes), vc, un[s] + c * k);
    }
  }
}

// The whole epilogue with the loads and the stores issued by every lane
// (vc_all: the point's offset, or beyond the buffer for inactive lanes,
// which then read 0 and whose stores are dropped, without traffic); the
// numbers of loads and stores a wave issues are then exactly
// epilogue_loads(stage) and epilogue_stores(stage).  Each stage has its own
// path, loads and stores together, so that no path leaves a load pending
// that the compiler would wait for where its register is next written.
template <typename T>
__device__ __forceinline__ void epilogue_all(const Patch& P, int stage,
                                             const T (&r)[NSLOT],
                                             uint32_t vc_all, int32_t nbytes) {
  double un[NSLOT], ac[NSLOT];
  if (stage == ST_RHS) {
    epilogue_store<T>(P, ST_RHS, r, vc_all, nbytes, un, ac);
  } else if (stage == ST_0) {
    epilogue_load(P, ST_0, vc_all, nbytes, un, ac);
    BSSN_PHASE();  // loads above, stores below
    epilogue_store<T>(P, ST_0, r, vc_all, nbytes, un, ac);
  } else if (stage == ST_3) {
    epilogue_load(P, ST_3, vc_all, nbytes, un, ac);
    BSSN_PHASE();
    epilogue_store<T>(P, ST_3, r, vc_all, nbytes, un, ac);
  } else if (stage == ST_1) {
    epilogue_load(P, ST_1, vc_all, nbytes, un, ac);
    BSSN_PHASE();
    epilogue_store<T>(P, ST_1, r, vc_all, nbytes, un, ac);
  } else {
    epilogue_load(P, ST_2, vc_all, nbytes, un, ac);
    BSSN_PHASE();
    epilogue_store<T>(P, ST_2, r, vc_all, nbytes, un, ac);
  }
}

template <typename T>
__device__ __forceinline__ void epilogue(const Patch& P, int stage,
                                         const T (&r)[NSLOT], uint32_t vc,
                                         int32_t nbytes) {
  double un[NSLOT], ac[NSLOT];
  epilogue_load(P, stage, vc, nbytes, un, ac);
  BSSN_PHASE();  // loads above, stores below
  epilogue_store<T>(P, stage, r, vc, nbytes, un, ac);
}

// One point of one patch: everything above, for the thread's point.
template <int ORDER, bool PERIODIC, typename T>
__device__ __forceinline__ void stage_point(const Patch& P, const Gauge& G,
                                            int stage, int x, int y, int z) {
  constexpr int R = FD<ORDER>::R;
  const int g = P.ghost;
  const int32_t nbytes = int32_t(P.sf * 8);
  const uint32_t sy8 = uint32_t(P.sy) * 8u, sz8 = uint32_t(P.sz) * 8u;
  const uint32_t vc =
      uint32_t(z + g) * sz8 + uint32_t(y + g) * sy8 + uint32_t(x + g) * 8u;
  const double xc = P.origin[0] + x * P.h[0];
  const double yc = P.origin[1] + y * P.h[1];
  const double zc = P.origin[2] + z * P.h[2];
  T r[NSLOT];
  if constexpr (!PERIODIC) {
    LdStatic<R> ld;
    ld.u = P.u_s;
    ld.sf = P.sf;
    ld.nbytes = nbytes;
    ld.vlo = vc - uint32_t(R) * (8u + sy8 + sz8);
    ld.str[0] = 8u;
    ld.str[1] = sy8;
    ld.str[2] = sz8;
    point_rhs<ORDER, T>(ld, P, xc, yc, zc, G, r);
  } else {
    LdPeriodic<R> ld;
    ld.u = P.u_s;
    ld.sf = P.sf;
    ld.nbytes = nbytes;
    const int pos[3] = {x, y, z};
    const uint32_t st[3] = {8u, sy8, sz8};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int k = -R; k <= R; ++k) {
        int q = pos[a] + k;
        q = q < 0 ? q + P.n[a] : (q >= P.n[a] ? q - P.n[a] : q);
        ld.o[a][R + k] = uint32_t(q + g) * st[a];
      }
    point_rhs<ORDER, T>(ld, P, xc, yc, zc, G, r);
  }
  epilogue<T>(P, stage, r, vc, nbytes);
}

// The point (x, y, z) of a workgroup-shaped tile; TILES selects which tiles
// a mixed-precision kernel of a pair takes (the predicate is uniform over
// the workgroup).
template <int ORDER, bool PERIODIC, int TILES>
__device__ __forceinline__ void stage_block(const Patch& P, const Gauge& G,
                                            const int stage, int x, int y,
                                            int z) {
  const bool active = x < P.n[0] && y < P.n[1];
  if constexpr (TILES != TILE_ALL) {
    const int g = P.ghost;
    const uint32_t vc = uint32_t(z + g) * uint32_t(P.sz) * 8u +
                        uint32_t(y + g) * uint32_t(P.sy) * 8u +
                        uint32_t(x + g) * 8u;
    const bool f64 =
        tile_needs_fp64(P, active, vc, int32_t(P.sf * 8), G.alpha_thr);
    if (f64 != (TILES == TILE_FP64)) return;
  }
  if (!active) return;
  if constexpr (TILES == TILE_FP32)
    stage_point<ORDER, PERIODIC, float>(P, G, stage, x, y, z);
  else
    stage_point<ORDER, PERIODIC, double>(P, G, stage, x, y, z);
}

// One patch: block (bx, by) of z-plane z covers x in [bx*BX, bx*BX + BX).
template <int ORDER, bool PERIODIC, int TILES>
__global__ void __launch_bounds__(256)
    k_stage(const Patch P, const Gauge G, const int stage) {
  stage_block<ORDER, PERIODIC, TILES>(
      P, G, stage, blockIdx.x * blockDim.x + threadIdx.x,
      blockIdx.y * blockDim.y + threadIdx.y, blockIdx.z);
}

// Many static patches: block b takes work item b = (patch, x0, y0, z0) and
// marches through planes z0 .. z0 + depth - 1 (those inside the patch), so
// the z-neighbour rows of its stencils are hits in the caches.
template <int ORDER, int TILES>
__global__ void __launch_bounds__(256)
    k_stage_direct_batch(const Patch* __restrict__ patches,
                         const DirectItem* __restrict__ work, const Gauge G,
                         const int stage, const int depth) {
  const DirectItem w = work[blockIdx.x];
  const Patch P = patches[w.patch];
  for (int dz = 0; dz < depth; ++dz) {
    const int z = w.z0 + dz;
    if (z >= P.n[2]) break;  // uniform over the workgroup
    stage_block<ORDER, false, TILES>(P, G, stage, w.x0 + threadIdx.x,
                                     w.y0 + threadIdx.y, z);
  }
}

// The right-hand side (FP64) at the outermost layer of interior points of a
// static patch (the points whose stencils reach a ghost layer first): the
// inward roots of the radiative boundary.  One thread per shell point,
// numbered as the two end planes in z (whole), then in the other planes
// the two end rows in y (whole), then the two ends of the remaining rows
// (ends that coincide on a one-point-wide axis are taken once).
struct ShellCount {
  int64_t na, nb, nc;
};
__host__ __device__ inline ShellCount shell_count(const int32_t (&n)[3]) {
  const int64_t nx = n[0], ny = n[1], nz = n[2];
  const int64_t nzp = nz > 1 ? 2 : 1, nyr = ny > 1 ? 2 : 1,
                nxe = nx > 1 ? 2 : 1;
  const int64_t nzi = nz > 2 ? nz - 2 : 0, nyi = ny > 2 ? ny - 2 : 0;
  return {nzp * nx * ny, nzi * nyr * nx, nzi * nyi * nxe};
}

template <int ORDER>
__global__ void __launch_bounds__(256) k_shell_rhs(const Patch P,
                                                   const Gauge G) {
  const int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const ShellCount c = shell_count(P.n);
  const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
  int x, y, z;
  if (t < c.na) {
    const int64_t pl = t / (int64_t(nx) * ny), m = t % (int64_t(nx) * ny);
    z = pl == 0 ? 0 : nz - 1;
    y = int(m / nx);
    x = int(m % nx);
  } else if (t < c.na + c.nb) {
    const int64_t u = t - c.na, row = u / nx;
    const int nyr = ny > 1 ? 2 : 1;
    x = int(u % nx);
    z = 1 + int(row / nyr);
    y = row % nyr == 0 ? 0 : ny - 1;
  } else if (t < c.na + c.nb + c.nc) {
    const int64_t u = t - c.na - c.nb;
    const int nxe = nx > 1 ? 2 : 1;
    const int64_t row = u / nxe;
    x = u % nxe == 0 ? 0 : nx - 1;
    y = 1 + int(row % (ny - 2));
    z = 1 + int(row / (ny - 2));
  } else {
    return;
  }
  stage_point<ORDER, false, double>(P, G, ST_RHS, x, y, z);
}

template <int ORDER>
hipError_t launch_shell_rhs_t(const Patch& P, const Gauge& G, hipStream_t st) {
  const ShellCount c = shell_count(P.n);
  const int64_t blocks = (c.na + c.nb + c.nc + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_shell_rhs<ORDER>), dim3(unsigned(blocks)), dim3(256),
                     0, st, P, G);
  return hipGetLastError();
}

// ---- host-side launch -------------------------------------------------------------
// Workgroup shape of the direct kernel: bx x (256 / bx); bx = 0 picks it
// from the patch width.
inline void stage_tile_shape(const Patch& P, int bx, dim3& blk) {
  if (bx <= 0) bx = P.n[0] > 32 ? 64 : 32;
  blk = dim3(bx, 256 / bx, 1);
}

template <int ORDER, bool PERIODIC>
hipError_t launch_stage_variant(const Patch& P, const Gauge& G, int stage,
                                int precision, int bx, hipStream_t st) {
  dim3 blk;
  stage_tile_shape(P, bx, blk);
  dim3 grd((P.n[0] + blk.x - 1) / blk.x, (P.n[1] + blk.y - 1) / blk.y, P.n[2]);
  if (precision == 0) {
    hipLaunchKernelGGL((k_stage<ORDER, PERIODIC, TILE_ALL>), grd, blk, 0, st,
                       P, G, stage);
  } else {
    hipLaunchKernelGGL((k_stage<ORDER, PERIODIC, TILE_FP32>), grd, blk, 0, st,
                       P, G, stage);
    hipLaunchKernelGGL((k_stage<ORDER, PERIODIC, TILE_FP64>), grd, blk, 0, st,
                       P, G, stage);
  }
  return hipGetLastError();
}

template <int ORDER>
hipError_t launch_direct_batch(const Patch* patches, const DirectItem* work,
                               int nwork, int bx, int depth, const Gauge& G,
                               int stage, int precision, hipStream_t st) {
  const dim3 blk(bx, 256 / bx, 1);
  if (precision == 0) {
    hipLaunchKernelGGL((k_stage_direct_batch<ORDER, TILE_ALL>), dim3(nwork),
                       blk, 0, st, patches, work, G, stage, depth);
  } else {
    hipLaunchKernelGGL((k_stage_direct_batch<ORDER, TILE_FP32>), dim3(nwork),
                       blk, 0, st, patches, work, G, stage, depth);
    hipLaunchKernelGGL((k_stage_direct_batch<ORDER, TILE_FP64>), dim3(nwork),
                       blk, 0, st, patches, work, G, stage, depth);
  }
  return hipGetLastError();
}

}  // namespace bssn
