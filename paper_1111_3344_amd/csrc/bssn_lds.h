// bssn_lds.h -- the fused RHS + RK4 stage as a persistent kernel that
// stages every slot's stencil box in LDS through the buffer->LDS DMA path.
//
// A workgroup of 256 threads owns one 16 x 4 x 4 tile at a time (one thread
// per point, wave w = z-plane w of the tile).  The point function visits the
// 25 slots one phase at a time (kPhaseSlot order); for each phase the haloed
// box of that slot, (16 + 2R + 1) x (4 + 2R) x (4 + 2R) doubles with rows
// starting one column early so that every 16-byte granule is aligned, sits
// in one of NBUF LDS buffers.  Boxes are fetched with
// buffer_load_dwordx4 ... lds (each lane moves one granule straight into
// LDS, no registers), NBUF - 1 phases ahead of use, and the pipeline runs
// on across tile boundaries, so the HBM/L2 latency of one phase hides behind
// the arithmetic of the previous ones.  Stencil taps are then ds_read_b64 /
// ds_read2_b64 with immediate offsets from one per-thread address.  Where
// it measured faster, granules a slot's stencils never read are not
// fetched (their lanes get an offset beyond the slot).
//
// Synchronisation per phase: wait until this wave's DMA for the phase has
// landed (an explicit vmcnt: the number of memory instructions the wave
// issued after it), barrier (all waves' granules have landed, and every
// wave is done with the previous phase's buffer), then issue the DMA for
// phase p + NBUF - 1 into the buffer phase p - 1 used.
//
// The epilogue (acc and the stage output) uses non-temporal buffer stores;
// in the order-4 FP64 kernel its loads are issued three phases before the
// end of the point function.
//
// Mixed precision runs as two launches per stage: k_stage_lds_f32 holds
// only the FP32 point function (at order 4 with a ring of three boxes, so
// that two workgroups share a CU) and skips the tiles whose minimum lapse
// is below the threshold; k_stage_lds_f64tiles then finds those tiles by
// the same test and runs them in FP64.
//
// Tiles are walked persistently (Walk): in blocks of 32 (or 64) tiles per
// XCD stepping together in z where the tile grid allows, else in contiguous
// z-column runs, so tiles whose halos overlap are in flight on one XCD and
// meet in its L2.
#pragma once
#include <hip/hip_runtime.h>

#include "bssn_stage.h"

namespace bssn {

template <int ORDER>
struct TileGeo;
// Box and ring geometry.  A box of G 16-byte granules is moved by NI DMA
// instructions of 64 lanes, at most L per wave (waves 0..2 issue L, the last
// wave the rest, NI - 3L); a buffer holds exactly NI * 64 granules.
// Mixed second derivatives (SHMIX): the inner first-difference sums of the
// tile's mixed stencils are formed once per position and shared through a
// scratch array of MIXD doubles (MX is the reach of the centred stencils).
// Order 4 has LDS to spare: every wave issues L instructions (the box is
// padded to 4L), and its mixed stencils (2 x 2 inner sums per pair) are too
// short for the shared scheme's extra barrier to pay (measured 14% slower
// on the 256^3 grid).
template <>
struct TileGeo<4> {
  static constexpr int R = 3, MX = 2, TX = 16, TY = 4, TZ = 4;
  static constexpr int W = 24;  // (TX + 2R + 1) rounded up to even
  static constexpr int H = TY + 2 * R, D = TZ + 2 * R;
  static constexpr int G = W * H * D / 2;    // granules per box
  static constexpr int L = (G + 255) / 256;  // DMA instructions per wave
  static constexpr int NI = 4 * L;           // DMA instructions per box
  static constexpr int NBUF = 5;             // ring of boxes in LDS; it
                                             // divides NSLOT, so every
                                             // phase's buffer is static
  static constexpr int BUFD = NI * 64 * 2;   // doubles per buffer
  static constexpr bool EARLY_EPI = true;    // epilogue loads at kEpiSlot
  static constexpr bool SHMIX = false;
};
// Order 8: the ring of three boxes and the centre block leave 8 KB of the
// 160 KB; trimming each buffer to the NI = 43 instructions its box needs
// (instead of 44) makes room for the mixed-derivative scratch, which
// removes 3/4 of the mixed stencils' LDS reads and a quarter of the FP64
// instructions.
template <>
struct TileGeo<8> {
  static constexpr int R = 5, MX = 4, TX = 16, TY = 4, TZ = 4;
  static constexpr int W = 28;
  static constexpr int H = TY + 2 * R, D = TZ + 2 * R;
  static constexpr int G = W * H * D / 2;
  static constexpr int NI = (G + 63) / 64;
  static constexpr int L = (NI + 3) / 4;
  static constexpr int NBUF = 3;
  static constexpr int BUFD = NI * 64 * 2;
  static constexpr bool EARLY_EPI = false;  // no registers to hold them
  static constexpr bool SHMIX = true;
};

// Layout of the shared mixed-derivative scratch (elements of the point
// function's type): PX, the y-sums at the tile's positions extended by MX
// in x ([TZ][TY][TX + 2 MX]); QX, the z-sums at the same positions; PZ, the
// y-sums at the tile's x, y positions on the MX planes below and above the
// tile ([2 MX][TY][TX]).  Every part is a whole number of 64-entry chunks.
template <class Geo>
struct MixGeo {
  static constexpr int M = Geo::MX, XW = Geo::TX + 2 * M;
  static constexpr int NX = Geo::TZ * Geo::TY * XW;  // entries of PX (QX)
  static constexpr int NZ = 2 * M * Geo::TY * Geo::TX;
  static constexpr int NE = 2 * NX + NZ;
  static constexpr int NC = NE / 64;          // chunks
  static constexpr int NR = (NC + 3) / 4;     // chunks per wave (at most)
  static_assert(NX % 64 == 0 && NZ % 64 == 0, "whole chunks per part");
};

// The same box geometry with a ring of NB buffers.
template <class Base, int NB>
struct GeoRing : Base {
  static constexpr int NBUF = NB;
};
// FP32 tiles of the split mixed stage: at order 4 a ring of 3 boxes keeps
// the workgroup within 80 KB of LDS, so two of them share a CU (the FP32
// point function fits the 256 registers that takes; the FP64 one does not).
template <int ORDER>
using GeoF32 = GeoRing<TileGeo<ORDER>, 3>;
// doubles of mixed-derivative scratch a kernel with geometry Geo declares
template <class Geo>
constexpr int mix_doubles() {
  return Geo::SHMIX ? MixGeo<Geo>::NE : 2;
}

static_assert(TileGeo<4>::TX == kLdsTile[0] && TileGeo<4>::TY == kLdsTile[1] &&
                  TileGeo<4>::TZ == kLdsTile[2] &&
                  TileGeo<8>::TX == kLdsTile[0] &&
                  TileGeo<8>::TY == kLdsTile[1] && TileGeo<8>::TZ == kLdsTile[2],
              "host work lists assume the kLdsTile shape");

typedef __attribute__((address_space(3))) void* lds_ptr_t;
typedef __attribute__((address_space(3))) double lds_double;

// LDS buffers of one workgroup.
template <class Geo>
struct LdsBufs {
  double* b[Geo::NBUF];
};

// Per-lane part of the DMA byte offsets (within one slot) of the granules
// this lane moves: the granule's place in the box, independent of the tile.
// The tile adds a wave-uniform byte offset (dma_tile_base), so one set of
// per-lane registers serves every tile.
template <class Geo>
__device__ __forceinline__ void dma_lane_offsets(const Patch& P, int wave,
                                                 int lane,
                                                 uint32_t (&off)[Geo::L]) {
#pragma unroll
  for (int j = 0; j < Geo::L; ++j) {
    const int q = (wave * Geo::L + j) * 64 + lane;
    const int col = q % (Geo::W / 2);
    const int row = q / (Geo::W / 2);
    const int yy = row % Geo::H, zz = row / Geo::H;
    const int64_t e = int64_t(zz) * P.sz + int64_t(yy) * P.sy + 2 * col;
    // Padding lanes (granules past the box) take an offset at or beyond
    // 2^31, so that with any tile base below 2^31 the sum stays out of the
    // slot (slots are < 2^31 bytes): their granules fill the buffer's pad
    // with zeros, without traffic.
    off[j] = q < Geo::G ? uint32_t(e * 8) : 0x80000000u;
  }
}

// Byte offset of the box origin (x0 - R - 1, y0 - R, z0 - R) of the tile
// at interior coordinates (x0, y0, z0), uniform over the workgroup.  The
// one box that starts 8 bytes before the slot (ghost = R, grid corner) has
// base 2^32 - 8: its first granule's first element (the alignment column,
// never read) is out of range, and its second element wraps to offset 0,
// the slot's first element, which it is.
template <class Geo>
__device__ __forceinline__ uint32_t dma_tile_base(const Patch& P, int x0,
                                                  int y0, int z0) {
  const int g = P.ghost;
  const int64_t e = int64_t(z0 + g - Geo::R) * P.sz +
                    int64_t(y0 + g - Geo::R) * P.sy + (x0 + g - Geo::R - 1);
  return __builtin_amdgcn_readfirstlane(uint32_t(e * 8));
}

// One buffer->LDS DMA instruction: every lane moves the 16 bytes at
// `voff` of the buffer described by (base, nbytes) to LDS address
// lds + 16 * lane.  Issued through inline asm so that the compiler's
// conservative LDS-DMA tracking (which cannot tell our ring buffers apart
// once the read pointer is opaque) does not insert vmcnt(0) before every LDS
// read; all waits for these transfers are explicit (pipeline_wait).  The
// instruction writes no register; M0 is set inside the block, with the one
// wait state the M0 -> LDS-DMA dependency needs.
typedef int v4i __attribute__((ext_vector_type(4)));
__device__ __forceinline__ v4i dma_rsrc(const double* base, int32_t nbytes) {
  const uint64_t a = reinterpret_cast<uint64_t>(base);
  v4i r;
  r.x = int(uint32_t(a));
  r.y = int(uint32_t(a >> 32) & 0xffffu);  // stride 0
  r.z = nbytes;
  r.w = kRsrcWord3;
  return r;
}
__device__ __forceinline__ void dma16(v4i r, uint32_t voff, uint32_t lds) {
  // the LDS address is uniform; say so, so that it stays in an SGPR even
  // where a uniform branch around the call hides that from the compiler
  lds = __builtin_amdgcn_readfirstlane(lds);
  asm volatile(
      "s_mov_b32 m0, %2\n\t"
      "s_nop 0\n\t"
      "buffer_load_dwordx4 %0, %1, 0 offen lds"
      :
      : "v"(voff), "s"(r), "s"(lds)
      : "memory", "m0");
}
__device__ __forceinline__ uint32_t lds_addr(const void* p) {
  return uint32_t(reinterpret_cast<uintptr_t>(
      (const __attribute__((address_space(3))) char*)(p)));
}
// (opaque base and stride, as for slot_rsrc)
__device__ __forceinline__ v4i slot_dma_rsrc(const double* u, int64_t sf,
                                             int s, int32_t nbytes) {
  const double* b = u;
  int64_t o = sf;
  asm volatile("" : "+s"(b), "+s"(o));
  return dma_rsrc(b + s * o, nbytes);
}

// Slots whose stencils include mixed second derivatives (gt_ij, phi,
// alpha, beta^i); the others only read the three axis lines through each
// point.
__host__ __device__ constexpr bool needs_mixed(int slot) {
  return (slot >= GXX && slot <= GZZ) || slot == PHI || slot == ALP ||
         (slot >= BETX && slot <= BETZ);
}

// Per-lane mask of the box granules this lane's DMA instructions move that
// a slot's stencils never read: bit j (star-only slots) or 16 + j (slots
// with mixed derivatives) for instruction j.  Star stencils read whole
// rows through the tile (y and z both in the tile), and the tile's x range
// of rows with y or z in the tile; mixed derivatives also read every row
// with y or z in the tile, and the tile's x range of the other rows.  The
// mask depends only on the lane, not on the tile.
template <class Geo>
__device__ __forceinline__ uint32_t dma_skip_mask(int wave, int lane) {
  uint32_t m = 0;
#pragma unroll
  for (int j = 0; j < Geo::L; ++j) {
    const int q = (wave * Geo::L + j) * 64 + lane;
    const int col = q % (Geo::W / 2);
    const int row = q / (Geo::W / 2);
    const int yy = row % Geo::H, zz = row / Geo::H;
    const bool in_y = yy >= Geo::R && yy < Geo::R + Geo::TY;
    const bool in_z = zz >= Geo::R && zz < Geo::R + Geo::TZ;
    // box column 0 is x0 - R - 1; the tile's x range is columns R+1 .. R+TX
    const bool in_x = 2 * col + 1 >= Geo::R + 1 && 2 * col <= Geo::R + Geo::TX;
    const bool star = (in_y && in_z) || ((in_y || in_z) && in_x);
    const bool mix = in_y || in_z || in_x;
    if (!star) m |= 1u << j;
    if (!mix) m |= 1u << (16 + j);
  }
  return m;
}

// The DMA of slot `slot`'s box into buf; granules the slot never reads get
// an offset beyond the slot (no traffic; their LDS words are not read).
template <class Geo>
__device__ __forceinline__ void dma_issue(const Patch& P, int slot,
                                          double* buf, int wave,
                                          const uint32_t (&off)[Geo::L],
                                          uint32_t tbase, uint32_t skip) {
  static_assert(Geo::L <= 16, "skip mask holds 16 instructions per kind");
  const v4i r = slot_dma_rsrc(P.u_s, P.sf, slot, int32_t(P.sf * 8));
  const uint32_t l0 = lds_addr(buf) + uint32_t(wave * Geo::L) * 1024u;
  const int sh = needs_mixed(slot) ? 16 : 0;
  // the last wave has NI - 3L instructions
  const bool last = __builtin_amdgcn_readfirstlane(wave) == 3;
#pragma unroll
  for (int j = 0; j < Geo::L; ++j) {
    if (Geo::NI < 4 * Geo::L && j >= Geo::NI - 3 * Geo::L && last) continue;
    const uint32_t o =
        (off[j] + tbase) | ((skip << (31 - (sh + j))) & 0x80000000u);
    dma16(r, o, l0 + j * 1024u);
  }
}

// Centre values the algebra needs before the slot's own phase (gt_ij,
// beta^i, alpha at phase 0) come from a per-tile LDS block (10 slots x 256
// points) that is fetched by DMA one tile ahead, at phase kCentrePhase of
// the previous tile, right after phase 0 read it; ordinary global loads
// would make the in-order vmcnt wait for every prefetch issued before them.
// Other centre values are taken from the slot's own box in its phase.
constexpr int kNCentre = 10;
constexpr int kCentreSlots[kNCentre] = {GXX,  GXY,  GXZ,  GYY, GYZ,
                                        GZZ,  BETX, BETY, BETZ, ALP};
__host__ __device__ constexpr int centre_index(int slot) {
  return slot <= GZZ && slot >= GXX     ? slot - GXX
         : slot >= BETX && slot <= BETZ ? 6 + slot - BETX
                                        : 9;
}
constexpr int kCentrePhase = 1;
constexpr int kCentreL = kNCentre * 128 / 256;  // DMA instructions per wave

// Per-lane DMA offsets of the centre block of the tile at (x0, y0, z0):
// instruction j of wave w moves half of slot kCentreSlots[(9w + j) / 2].
__device__ __forceinline__ void centre_dma(const Patch& P, double* sc,
                                           int x0, int y0, int z0, int wave,
                                           int lane) {
  const int g = P.ghost;
#pragma unroll
  for (int j = 0; j < kCentreL; ++j) {
    const int ins = wave * kCentreL + j;
    const int slot = kCentreSlots[ins >> 1];
    const int within = (ins & 1) * 64 + lane;
    const int row = within >> 3, col = within & 7;
    const int tz = row >> 2, ty = row & 3;
    const int64_t e = int64_t(z0 + tz + g) * P.sz + int64_t(y0 + ty + g) * P.sy +
                      (x0 + g) + 2 * col;
    dma16(slot_dma_rsrc(P.u_s, P.sf, slot, int32_t(P.sf * 8)),
          uint32_t(e * 8), lds_addr(sc) + uint32_t(ins) * 1024u);
  }
}

// s_waitcnt vmcnt(min(N + extra, 63)) lgkmcnt(0) for extra a multiple of
// NSLOT (0 .. 4 NSLOT), rounded down to a value that is never above the
// true count.
template <int N>
__device__ __forceinline__ void vm_wait_n() {
  asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)" ::"n"(N < 63 ? N : 63)
               : "memory");
}
template <int N>
__device__ __forceinline__ void vm_wait_extra(int extra) {
  if (extra <= 0)
    vm_wait_n<N>();
  else if (extra < 2 * NSLOT)
    vm_wait_n<N + NSLOT>();
  else
    vm_wait_n<N + 2 * NSLOT>();
}

// The slot whose phase issues the epilogue loads early: the first of the
// last three phases (the shift), after which only their stencils and a
// short stretch of algebra remain.
constexpr int kEpiSlot = BETX;

// Box element of the lowest tap (y - M for y sums, z - M for z sums) of
// entry `lane` of chunk c of the shared mixed-derivative scratch (MixGeo
// layout).  c is uniform over the wave; the three kinds of chunk (PX, QX,
// PZ) take separate code, so that where c is known at compile time only
// one remains.
template <class Geo>
__device__ __forceinline__ int mix_entry(int c, int lane) {
  using MG = MixGeo<Geo>;
  constexpr int M = MG::M, XW = MG::XW, R = Geo::R, W = Geo::W, H = Geo::H;
  if (c < 2 * MG::NX / 64) {  // PX (y sums) or QX (z sums), x-extended
    // entry i = q XW + ix with q = tz TY + ty: its box element is
    // tz (H W) + ty W + ix + const = tz (H - TY) W + q (W - XW) + i + const
    const bool qx = c >= MG::NX / 64;
    const unsigned i =
        unsigned((qx ? c - MG::NX / 64 : c) * 64) + unsigned(lane);
    const unsigned q = i / unsigned(XW), tz = q / unsigned(Geo::TY);
    constexpr int C0 = (R * H + R - M) * W + R + 1 - M;  // PX: (R, R - M)
    constexpr int C1 = ((R - M) * H + R) * W + R + 1 - M;  // QX: (R - M, R)
    return int(tz * unsigned((H - Geo::TY) * W) + q * unsigned(W - XW) + i) +
           (qx ? C1 : C0);
  }
  // PZ: y sums on the planes beyond the tile; a chunk is one plane
  static_assert(Geo::TX * Geo::TY == 64, "one PZ plane per chunk");
  const int pz = c - 2 * MG::NX / 64;
  const int zr = pz < M ? pz - M : Geo::TZ + pz - M;
  return ((zr + R) * H + (lane >> 4) + R - M) * W + (lane & 15) + R + 1;
}

// Distinct empty asm at both ends of each code path of a uniform branch,
// so that the compiler keeps the paths apart (each with its own immediate
// LDS offsets) instead of merging them into one with selected addresses.
template <int K>
__device__ __forceinline__ void path_mark();
template <>
__device__ __forceinline__ void path_mark<0>() {
  asm volatile("; path 0");
}
template <>
__device__ __forceinline__ void path_mark<1>() {
  asm volatile("; path 1");
}

// Loader used by point_rhs inside the pipelined kernel.  Phase p of the
// k-th tile of a workgroup is global phase k*NSLOT + p and uses ring buffer
// (k*NSLOT + p) mod NBUF.
template <class Geo, bool EARLY, bool CORNER>
struct LdLds {
  const Patch* P;
  double* ring;            // NBUF buffers of BUFD doubles
  double* sc;              // centre block
  const uint32_t* off;     // per-lane DMA offsets within a box
  uint32_t tb_cur, tb_nxt;  // box base of this tile and of the next one
  int nxt[3];              // next tile's origin (centre block prefetch)
  int pbase;               // (k * NSLOT) mod NBUF
  int wave, lane, tid;
  uint32_t skip;           // dma_skip_mask of this lane
  int cidx;                // element index in a box of the thread's centre
                           // or (CORNER) of its stencil corner
                           // (x-R, y-R, z-R)
  // early epilogue loads: issued when the phase of kEpiSlot starts (the
  // algebra left after it gives their latency something to hide behind)
  int stage;
  uint32_t vc_epi;         // byte offset of the point, or out of range
  int32_t nbytes;
  int epi_loads;           // loads issued this way at this tile (per wave)
  int prev_loads;          // the same for the previous tile (0 at the first)
  int prev_stores;         // stores of the previous tile's epilogue in this
                           // wave (0 at the first tile)
  mutable double un[NSLOT], ac[NSLOT];
  // this thread's cidx in the current phase's buffer; set per phase
  // through an opaque move so the compiler derives every tap from this one
  // register with immediate offsets instead of hoisting (and spilling) a
  // base address per buffer out of the tile loop
  mutable const lds_double* pc;
  // shared mixed derivatives: the current phase's box, the scratch array
  // and this lane's entry positions in a box (lowest tap, elements)
  mutable const lds_double* box;
  void* mix;
  static constexpr bool kSharedMixed = Geo::SHMIX;

  __device__ __forceinline__ double* buffer(int p) const {
    return ring + ((pbase + p) % Geo::NBUF) * Geo::BUFD;
  }
  __device__ __forceinline__ double g(int s) const {
    return ((const lds_double*)sc)[centre_index(s) * 256 + tid];
  }
  __device__ __forceinline__ void enter(int s) const {
    const int p = phase_of(s);
    if (p != 0) phase(p);  // the kernel runs phase 0 itself
    if (EARLY && s == kEpiSlot)
      epilogue_load(*P, stage, vc_epi, nbytes, un, ac);
    const lds_double* b = (const lds_double*)buffer(p) + cidx;
    asm volatile("" : "+v"(b));
    pc = b;
    if constexpr (Geo::SHMIX) box = (const lds_double*)buffer(p);
  }
  // one pipeline step at phase p (0 <= p < NSLOT)
  __device__ __forceinline__ void phase(int p) const {
    // Wait until this wave's DMA for phase p has landed.  vmcnt counts
    // this wave's memory instructions in issue order, so the count to wait
    // for is the number issued after that DMA: the prefetches of phases
    // p+1 .. p+NBUF-2; for phases 2 .. NBUF the centre block issued at
    // phase 1; after the phase of kEpiSlot, the early epilogue loads; and
    // at phases 0 .. NBUF-2 of every tile but the first, the previous
    // tile's epilogue stores, plus its early loads where they followed the
    // DMA (issued at phase NSLOT + p - NBUF + 1 of that tile).  The field
    // holds at most 63, and waiting for fewer than that number is always
    // correct.  lgkmcnt(0): this wave's reads of the buffer about to be
    // refilled have completed.
    // (without early loads, PE = NSLOT: the loads come with the stores)
    constexpr int PE = EARLY ? phase_of(kEpiSlot) : NSLOT;
    int extra = 0;
    if (p > PE) extra = epi_loads;
    if (p <= Geo::NBUF - 2)
      extra = prev_stores +
              (p <= PE - NSLOT + Geo::NBUF - 1 ? prev_loads : 0);
    // DMA instructions per phase: L, and NI - 3L in the last wave
    constexpr int L3 = Geo::NI - 3 * Geo::L;
    const bool centre = p > kCentrePhase && p <= kCentrePhase + Geo::NBUF - 1;
    if (wave == 3 && L3 < Geo::L) {
      if (centre)
        vm_wait_extra<(Geo::NBUF - 2) * L3 + kCentreL>(extra);
      else
        vm_wait_extra<(Geo::NBUF - 2) * L3>(extra);
    } else {
      if (centre)
        vm_wait_extra<(Geo::NBUF - 2) * Geo::L + kCentreL>(extra);
      else
        vm_wait_extra<(Geo::NBUF - 2) * Geo::L>(extra);
    }
    __builtin_amdgcn_s_barrier();
    const int q = p + Geo::NBUF - 1;  // phase to prefetch
    uint32_t o[Geo::L];
#pragma unroll
    for (int j = 0; j < Geo::L; ++j) o[j] = off[j];
    if (q < NSLOT)
      dma_issue<Geo>(*P, kPhaseSlot[q], buffer(q), wave, o, tb_cur, skip);
    else
      dma_issue<Geo>(*P, kPhaseSlot[q - NSLOT], buffer(q), wave, o, tb_nxt,
                     skip);
    if (p == kCentrePhase)
      centre_dma(*P, sc, nxt[0], nxt[1], nxt[2], wave, lane);
  }
  __device__ __forceinline__ int str(int a) const {
    return a == 0 ? 1 : (a == 1 ? Geo::W : Geo::W * Geo::H);
  }
  // With CORNER, pc is the thread's stencil corner, so every tap is a
  // non-negative immediate offset (fewer address adds, more ds_read2 pairs;
  // measured faster for the FP32 and the order-8 kernels, slower for the
  // order-4 FP64 one).
  static constexpr int kC =
      CORNER ? Geo::R * (1 + Geo::W + Geo::W * Geo::H) : 0;
  __device__ __forceinline__ double c(int) const { return pc[kC]; }
  __device__ __forceinline__ double ax(int, int a, int k) const {
    return pc[kC + k * str(a)];
  }
  __device__ __forceinline__ double pl(int, int a, int i, int b, int j) const {
    return pc[kC + i * str(a) + j * str(b)];
  }

  // The three mixed second derivatives of the current phase's slot at this
  // thread's point, as tensor products of the centred first-difference
  // stencil: d_x d_y u = sum_i a_i (Sy(x+i) - Sy(x-i)) with the inner sums
  // Sy(x') = sum_j a_j (u(x', y+j) - u(x', y-j)), likewise d_x d_z (inner z
  // sums at x-shifted points) and d_y d_z = d_z of the inner y sums.  Every
  // inner sum the tile needs is formed once by one lane (MixGeo layout),
  // written to LDS, and read back after a barrier by the lanes that need
  // it, instead of each lane forming the 2M inner sums of each pair itself.
  // Every wave calls it at the same phases (it holds a barrier).
  //
  // Addressing: the taps of an inner sum are read from one opaque VGPR base
  // with immediate offsets (a plain asm, so that it orders nothing else).
  // Latency: the taps of round r + 1 are read before the arithmetic of
  // round r, and the read-back taps of all three pairs before their sums.
  template <int ORDER, int S>
  __device__ __forceinline__ void entry_taps(const lds_double* b,
                                             double (&t)[8]) const {
    constexpr int M = FD<ORDER>::M;
    static_assert(2 * M == 8, "eight taps per inner sum");
    asm("" : "+v"(b));
#pragma unroll
    for (int j = 1; j <= M; ++j) {
      t[2 * j - 2] = b[(M + j) * S];
      t[2 * j - 1] = b[(M - j) * S];
    }
  }
  // Kind of the chunks of round RR (chunks 4 RR .. 4 RR + 3, one per wave):
  // 0 all z sums (QX), 1 all y sums (PX, PZ), 2 both (chosen per wave).
  template <int RR>
  static constexpr int round_kind() {
    using MG = MixGeo<Geo>;
    int nz = 0, ny = 0;
    for (int w = 0; w < 4; ++w) {
      const int c = 4 * RR + w;
      if (c >= MG::NX / 64 && c < 2 * MG::NX / 64)
        ++nz;
      else
        ++ny;
    }
    return ny == 0 ? 0 : (nz == 0 ? 1 : 2);
  }
  template <int ORDER, int RR>
  __device__ __forceinline__ void round_taps(int w, int ln,
                                             double (&t)[8]) const {
    using MG = MixGeo<Geo>;
    constexpr int SY = Geo::W, SZ = Geo::W * Geo::H, K = round_kind<RR>();
    const int c = 4 * RR + w;
    if constexpr (K == 0) {
      entry_taps<ORDER, SZ>(box + mix_entry<Geo>(c, ln), t);
    } else if constexpr (K == 1) {
      entry_taps<ORDER, SY>(box + mix_entry<Geo>(c, ln), t);
    } else if (c >= MG::NX / 64 && c < 2 * MG::NX / 64) {
      path_mark<0>();
      entry_taps<ORDER, SZ>(box + mix_entry<Geo>(c, ln), t);
      path_mark<0>();
    } else {
      path_mark<1>();
      entry_taps<ORDER, SY>(box + mix_entry<Geo>(c, ln), t);
      path_mark<1>();
    }
  }
  // Rounds RR .. NR - 1 of the inner sums; cur holds the taps of round RR.
  template <int ORDER, typename T, int RR>
  __device__ __forceinline__ void rounds(int w, int ln, double (&cur)[8],
                                         double (&nxt)[8]) const {
    using F = FD<ORDER>;
    using MG = MixGeo<Geo>;
    constexpr int M = F::M;
    typedef __attribute__((address_space(3))) T lds_t;
    if constexpr (RR + 1 < MG::NR) round_taps<ORDER, RR + 1>(w, ln, nxt);
    T v = T(0);
#pragma unroll
    for (int j = 1; j <= M; ++j)
      v += T(F::a(j)) * T(cur[2 * j - 2] - cur[2 * j - 1]);
    ((lds_t*)mix)[(4 * RR + w) * 64 + lane] = v;
    if constexpr (RR + 1 < MG::NR) rounds<ORDER, T, RR + 1>(w, ln, nxt, cur);
  }
  template <int ORDER, typename T>
  __device__ __forceinline__ void mixed3(T ihxy, T ihxz, T ihyz, T& dxy,
                                         T& dxz, T& dyz) const {
    using F = FD<ORDER>;
    using MG = MixGeo<Geo>;
    constexpr int M = MG::M, XW = MG::XW, NX = MG::NX;
    static_assert(MG::NC == 4 * MG::NR, "whole rounds of chunks");
    typedef __attribute__((address_space(3))) T lds_t;
    lds_t* mx = (lds_t*)mix;
    // the lane number through an opaque copy, so that the entry positions
    // are formed here rather than hoisted out of the tile loop (where they
    // would hold registers through every phase); the wave index masked to
    // its range, so that a round's chunk kind folds where it can
    int ln = lane;
    asm volatile("" : "+v"(ln));
    const int w = wave & 3;
    {
      double ta[8], tb[8];
      round_taps<ORDER, 0>(w, ln, ta);
      rounds<ORDER, T, 0>(w, ln, ta, tb);
    }
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    const int tx = ln & 15, ty = ln >> 4;
    // lowest x tap (x - M) of this point in PX and QX
    const lds_t* px = mx + (w * Geo::TY + ty) * XW + tx;
    asm("" : "+v"(px));
    // y sums at (x, y, z + k): PX inside the tile, PZ on the planes beyond
    const lds_t* pxc = mx + ty * XW + tx + M;
    const lds_t* pzc = mx + 2 * NX + ty * Geo::TX + tx;
    T ta[2 * M], tq[2 * M], td[2 * M];
#pragma unroll
    for (int i = 1; i <= M; ++i) {
      ta[2 * i - 2] = px[M + i];
      ta[2 * i - 1] = px[M - i];
      tq[2 * i - 2] = px[NX + M + i];
      tq[2 * i - 1] = px[NX + M - i];
      const int zp = w + i, zm = w - i;  // uniform
      td[2 * i - 2] = zp < Geo::TZ ? pxc[zp * Geo::TY * XW]
                                   : pzc[(zp - Geo::TZ + M) * Geo::TY * Geo::TX];
      td[2 * i - 1] = zm >= 0 ? pxc[zm * Geo::TY * XW]
                              : pzc[(zm + M) * Geo::TY * Geo::TX];
    }
    T a = T(0), q = T(0), d = T(0);
#pragma unroll
    for (int i = 1; i <= M; ++i) {
      a += T(F::a(i)) * (ta[2 * i - 2] - ta[2 * i - 1]);
      q += T(F::a(i)) * (tq[2 * i - 2] - tq[2 * i - 1]);
      d += T(F::a(i)) * (td[2 * i - 2] - td[2 * i - 1]);
    }
    dxy = a * ihxy;
    dxz = q * ihxz;
    dyz = d * ihyz;
    keep(dxy);
    keep(dxz);
    keep(dyz);
  }
};


// Tile walk.  Tiles are numbered z fastest within an (x, y) column:
// t = iz + ntz * (ix + ntx * iy).  Workgroup b owns the contiguous range of
// tiles [lo, hi) of position walk_pos(b) in an even split, so it marches
// along z through whole columns (consecutive boxes share 2R of their
// TZ + 2R planes, which the caches then serve), and the workgroups of one
// XCD (dispatched round-robin: b, b+8, ...) own neighbouring columns, whose
// x/y halos meet in that XCD's L2.
struct TileMap {
  int ntx, nty, ntz, ntiles;
  int bx, by, bz;  // block shape of the blocked walk, bx = 0: contiguous
};
__host__ __device__ __forceinline__ int walk_pos(int wg, int nwg) {
  return (nwg & 7) == 0 ? (wg & 7) * (nwg >> 3) + (wg >> 3) : wg;
}
__host__ __device__ __forceinline__ void walk_range(int lin, int nwg,
                                                    int ntiles, int& lo,
                                                    int& hi) {
  lo = int((int64_t(ntiles) * lin) / nwg);
  hi = int((int64_t(ntiles) * (lin + 1)) / nwg);
}

// Origin (interior coordinates) of tile t of the TileMap numbering.
__device__ __forceinline__ void tile_origin(int t, int ntx, int ntz, int& x0,
                                            int& y0, int& z0) {
  const int iz = t % ntz, col = t / ntz;
  x0 = (col % ntx) * kLdsTile[0];
  y0 = (col / ntx) * kLdsTile[1];
  z0 = iz * kLdsTile[2];
}

// The tiles one workgroup visits, in order (one walker type, so the
// right-hand side is inlined once).  Tile k is c = k / nk, kz = k mod nk:
//   contiguous walk (bx = 0): tiles tlo + k of the TileMap numbering
//     (z fastest within an (x, y) column); nk = count, c = 0;
//   blocked walk (single patches whose tile grid divides into blocks of
//     bx x by x bz = 32 tiles, or 64 with two workgroups per CU): the
//     workgroups of one XCD hold one tile each of a block, step through
//     the block's column together in z by
//     bz tiles, then move on to the XCD's next block (blocks c*8 + xcd).
//     Neighbouring tiles in x, y and z are then fetched at the same time on
//     one XCD, and between two z-steps the L2 only has to keep the overlap
//     planes of a (16 bx + 2R) x (4 by + 2R) footprint.
struct Walk {
  int n;            // tiles this workgroup visits
  int tlo, ntx, ntz;
  int lx, ly, lz;   // this workgroup's tile within a block
  int bx, by, bz;   // block shape in tiles (0: contiguous walk)
  int xcd, nrx, nk;
  __device__ __forceinline__ int count() const { return n; }
  __device__ __forceinline__ void origin(int k, int& x0, int& y0,
                                         int& z0) const {
    if (bx == 0) {
      tile_origin(tlo + k, ntx, ntz, x0, y0, z0);
    } else {
      const int r = xcd + 8 * (k / nk), kz = k % nk;
      x0 = ((r % nrx) * bx + lx) * kLdsTile[0];
      y0 = ((r / nrx) * by + ly) * kLdsTile[1];
      z0 = (kz * bz + lz) * kLdsTile[2];
    }
  }
};
__device__ __forceinline__ Walk walk_contig(int tlo, int n, int ntx,
                                            int ntz) {
  Walk w{};
  w.n = n;
  w.tlo = tlo;
  w.ntx = ntx;
  w.ntz = ntz;
  w.bx = 0;
  return w;
}

// Arithmetic of the tiles of an LDS kernel:
//   TP_F64   FP64 everywhere;
//   TP_F32   the FP32 launch of a mixed-precision stage: FP32 stencils and
//            algebra on every tile whose minimum lapse is at least
//            G.alpha_thr; a tile below it runs through the pipeline without
//            arithmetic and is left to the FP64 pass (k_stage_lds_f64tiles,
//            k_stage_lds_batch_f64tiles), which finds it by the same test.
enum : int { TP_F64 = 0, TP_F32 = 1 };

// Minimum lapse over the tile's points, taken from the centre block (which
// holds all 256 of them) in every wave, so that each wave reaches the same
// value without a barrier.  Points outside the grid do not count.  fmin is
// exact, so the value does not depend on the order of reduction;
// k_stage_lds_f64tiles computes the same minimum from global memory.
__device__ __forceinline__ double tile_lapse_min(const double* sc,
                                                 const Patch& P, int x, int y,
                                                 int z0, int lane) {
  const lds_double* sa = (const lds_double*)sc + centre_index(ALP) * 256;
  double a = 1.0e300;
  const bool in_xy = x < P.n[0] && y < P.n[1];
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const double v = sa[w * 64 + lane];
    if (in_xy && z0 + w < P.n[2]) a = fmin(a, v);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) a = fmin(a, __shfl_xor(a, off, 64));
  return a;
}

// The point function and epilogue of one thread's point in arithmetic T.
// KSH: a point on the outermost interior layer (shell) also stores its
// right-hand side to kout (the radiative boundary's roots, state layout);
// the stores follow the epilogue's.
template <int ORDER, typename T, bool EARLY, bool KSH, class LD>
__device__ __forceinline__ void tile_point(const LD& ld, const Patch& P,
                                           const Gauge& G, int stage,
                                           double xc, double yc, double zc,
                                           uint32_t vc, int32_t nbytes,
                                           bool active, bool shell,
                                           double* kout) {
  T r[NSLOT];
  point_rhs<ORDER, T>(ld, P, xc, yc, zc, G, r);
  if (EARLY) {
    if (active) epilogue_store<T>(P, stage, r, vc, nbytes, ld.un, ld.ac);
  } else {
    epilogue_all<T>(P, stage, r, ld.vc_epi, nbytes);
  }
  if constexpr (KSH) {
    if (active && shell) {
#pragma unroll
      for (int s = 0; s < NSLOT; ++s)
        bstore_nt(slot_rsrc(kout, P.sf, s, nbytes), vc, double(r[s]));
    }
  }
}

// The tiles Wk names, of patch P, pipelined through the workgroup's LDS
// ring (Geo: box and ring geometry; WK: a walk with count() and origin()).
// On return every DMA of this call has landed; the caller places a barrier
// before the ring is filled again.
template <int ORDER, int TP, bool TRIM, class Geo = TileGeo<ORDER>,
          class WK = Walk, bool KSH = false>
__device__ __forceinline__ void lds_tiles(const Patch& P, const Gauge& G,
                                          const int stage, const WK& Wk,
                                          double* ring, double* sc,
                                          double* mixs,
                                          double* kout = nullptr) {
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int tx = lane & 15, ty = lane >> 4, tz = wave;
  const int ntile_mine = Wk.count();
  if (ntile_mine <= 0) return;
  uint32_t off[Geo::L];
  dma_lane_offsets<Geo>(P, wave, lane, off);
  int x0, y0, z0, xn, yn, zn;
  Wk.origin(0, x0, y0, z0);
  uint32_t tbA = dma_tile_base<Geo>(P, x0, y0, z0);
  Wk.origin(ntile_mine > 1 ? 1 : 0, xn, yn, zn);
  uint32_t tbB = dma_tile_base<Geo>(P, xn, yn, zn);
  // TRIM: DMA only the granules each slot reads (the out-of-range lanes
  // still cost their address slot, and the mask costs a register)
  const uint32_t skip = TRIM ? dma_skip_mask<Geo>(wave, lane) : 0u;
  // prologue: centre block and phases 0 .. NBUF-2 of the first tile
  centre_dma(P, sc, x0, y0, z0, wave, lane);
#pragma unroll
  for (int q = 0; q < Geo::NBUF - 1; ++q)
    dma_issue<Geo>(P, kPhaseSlot[q], ring + q * Geo::BUFD, wave, off, tbA,
                   skip);

  const int32_t nbytes = int32_t(P.sf * 8);
  const uint32_t sy8 = uint32_t(P.sy) * 8u, sz8 = uint32_t(P.sz) * 8u;
  int prev_loads = 0, prev_stores = 0;  // this wave's last epilogue
  for (int k = 0; k < ntile_mine; ++k) {
    Wk.origin(k, x0, y0, z0);
    const int x = x0 + tx, y = y0 + ty, z = z0 + tz;
    const bool active = x < P.n[0] && y < P.n[1] && z < P.n[2];
    const bool shell = KSH && (x == 0 || y == 0 || z == 0 || x == P.n[0] - 1 ||
                               y == P.n[1] - 1 || z == P.n[2] - 1);
    const int g = P.ghost;
    // early epilogue loads where the registers allow (order 4, FP64);
    // corner-based tap addressing for the FP32 and order-8 kernels
    constexpr bool early = Geo::EARLY_EPI && TP == TP_F64;
    constexpr bool corner = TP == TP_F32 || ORDER == 8;
    LdLds<Geo, early, corner> ld;
    ld.P = &P;
    ld.ring = ring;
    ld.sc = sc;
    ld.mix = mixs;
    ld.off = off;
    ld.tb_cur = tbA;
    ld.tb_nxt = tbB;
    ld.nxt[0] = xn;
    ld.nxt[1] = yn;
    ld.nxt[2] = zn;
    ld.pbase = NSLOT % Geo::NBUF == 0 ? 0 : (k * NSLOT) % Geo::NBUF;
    ld.wave = wave;
    ld.lane = lane;
    ld.tid = tid;
    ld.skip = skip;
    ld.stage = stage;
    ld.nbytes = nbytes;
    ld.epi_loads = early ? epilogue_loads(stage) : 0;
    ld.prev_loads = prev_loads;
    ld.prev_stores = prev_stores;
    ld.cidx = (tz * Geo::H + ty) * Geo::W + tx + 1 +
              (corner ? 0 : Geo::R * (1 + Geo::W + Geo::W * Geo::H));
    const uint32_t vc = active ? uint32_t(z + g) * sz8 + uint32_t(y + g) * sy8 +
                                     uint32_t(x + g) * 8u
                               : 0u;
    // inactive lanes load from beyond the buffer: no traffic, value 0
    ld.vc_epi = active ? vc : 0xFFFFFFF0u;
    ld.phase(0);  // phase 0's box and this tile's centre block have landed
    const double xc = P.origin[0] + x * P.h[0];
    const double yc = P.origin[1] + y * P.h[1];
    const double zc = P.origin[2] + z * P.h[2];
    bool computed = true;
    if constexpr (TP == TP_F64) {
      tile_point<ORDER, double, early, KSH>(ld, P, G, stage, xc, yc, zc, vc,
                                            nbytes, active, shell, kout);
    } else {
      if (tile_lapse_min(sc, P, x, y, z0, lane) < G.alpha_thr) {
        // left to the FP64 pass: keep the pipeline going (waits, barriers,
        // prefetches) through the tile's other phases
#pragma unroll
        for (int p = 1; p < NSLOT; ++p) ld.phase(p);
        computed = false;
      } else {
        tile_point<ORDER, float, early, KSH>(ld, P, G, stage, xc, yc, zc, vc,
                                             nbytes, active, shell, kout);
      }
    }
    prev_loads =
        !computed ? 0 : (early ? ld.epi_loads : epilogue_loads(stage));
    // (without early loads every lane stores, inactive ones beyond the
    // buffer; with them only active lanes do, and a wave without any
    // issues none)
    prev_stores =
        computed && (!early || __builtin_amdgcn_ballot_w64(active) != 0)
            ? epilogue_stores(stage)
            : 0;
    // the shell stores of this wave, if any lane made them (a wave whose
    // lanes all skip them may still issue them with no lane enabled, which
    // only makes the next waits longer than needed)
    if (KSH && computed && __builtin_amdgcn_ballot_w64(active && shell) != 0)
      prev_stores += NSLOT;
    // next tile: its box base becomes current, prepare the one after
    tbA = tbB;
    if (k + 2 < ntile_mine) {
      Wk.origin(k + 2, xn, yn, zn);
      tbB = dma_tile_base<Geo>(P, xn, yn, zn);
    }
  }
  // drain outstanding DMA (the last tile prefetched a next one that is not
  // used) and this wave's LDS reads
  asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
}

// One patch: workgroup b takes the tiles of position walk_pos(b).
// The walk of workgroup blockIdx.x of a launch of nwg workgroups over M.
__device__ __forceinline__ Walk walk_of(const TileMap& M, int nwg) {
  Walk w{};
  if (M.bx > 0) {
    w.xcd = blockIdx.x & 7;
    const int l = blockIdx.x >> 3;
    w.lx = l % M.bx;
    w.ly = (l / M.bx) % M.by;
    w.lz = l / (M.bx * M.by);
    w.bx = M.bx;
    w.by = M.by;
    w.bz = M.bz;
    w.nrx = M.ntx / M.bx;
    w.nk = M.ntz / M.bz;
    const int nblk = w.nrx * (M.nty / M.by);
    w.n = (nblk > w.xcd ? (nblk - w.xcd + 7) / 8 : 0) * w.nk;
  } else {
    int tlo, thi;
    walk_range(walk_pos(blockIdx.x, nwg), nwg, M.ntiles, tlo, thi);
    w = walk_contig(tlo, thi - tlo, M.ntx, M.ntz);
  }
  return w;
}

// Stagger the workgroups' start over about one order-4 tile time (eight
// phases 3.4 us apart, spread over each XCD's CUs).  With equal work per
// tile the workgroups of a single-grid launch would otherwise stay in step
// and their epilogue bursts (all 25 slots loaded and stored at once) would
// meet in HBM.  Only where a workgroup has many tiles, so that the delay
// is small against its run.
__device__ __forceinline__ void stagger_start(int ntile_mine) {
  if (ntile_mine < 128) return;
  const int ph = (blockIdx.x >> 3) & 7;
  for (int i = 0; i < ph; ++i) __builtin_amdgcn_s_sleep(127);
}

// One patch, FP64: workgroup b takes the tiles of walk_of(b).  KSH: also
// the right-hand side at the outermost interior layer into kout.
template <int ORDER, bool KSH = false>
__global__ void __launch_bounds__(256)
    k_stage_lds(const Patch P, const Gauge G, const int stage,
                const TileMap M, double* const kout) {
  using Geo = TileGeo<ORDER>;
  __shared__ __attribute__((aligned(16))) double ring[Geo::NBUF * Geo::BUFD];
  __shared__ __attribute__((aligned(16))) double sc[kNCentre * 256];
  __shared__ __attribute__((aligned(16))) double mixs[mix_doubles<Geo>()];
  const Walk w = walk_of(M, gridDim.x);
  // order 4 only: 2% on a 256^3 grid; neutral at order 8
  if (ORDER == 4) stagger_start(w.count());
  // trimmed DMA: granules no stencil reads are not fetched (3-4% faster
  // at order 4 too since the DMA offsets became lane constants)
  lds_tiles<ORDER, TP_F64, true, TileGeo<ORDER>, Walk, KSH>(
      P, G, stage, w, ring, sc, mixs, kout);
}

// One patch, mixed precision, first launch: the FP32 tiles.  At order 4
// two workgroups share a CU (GeoF32 ring, at most 256 registers per lane).
template <int ORDER, bool KSH = false>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(ORDER == 4 ? 2 : 1,
                                       ORDER == 4 ? 2 : 1)))
    k_stage_lds_f32(const Patch P, const Gauge G, const int stage,
                    const TileMap M, double* const kout) {
  using Geo = GeoF32<ORDER>;
  __shared__ __attribute__((aligned(16))) double ring[Geo::NBUF * Geo::BUFD];
  __shared__ __attribute__((aligned(16))) double sc[kNCentre * 256];
  __shared__ __attribute__((aligned(16))) double mixs[mix_doubles<Geo>()];
  lds_tiles<ORDER, TP_F32, true, Geo, Walk, KSH>(
      P, G, stage, walk_of(M, gridDim.x), ring, sc, mixs, kout);
}

// Tiles named by an LDS list of tile numbers (TileMap numbering).
typedef __attribute__((address_space(3))) int lds_int;
struct ListWalk {
  const lds_int* t;
  int n, ntx, ntz;
  __device__ __forceinline__ int count() const { return n; }
  __device__ __forceinline__ void origin(int k, int& x0, int& y0,
                                         int& z0) const {
    tile_origin(t[k], ntx, ntz, x0, y0, z0);
  }
};

// One tile (TileMap numbering), its number held in a register.
struct OneWalk {
  int t, ntx, ntz;
  __device__ __forceinline__ int count() const { return 1; }
  __device__ __forceinline__ void origin(int, int& x0, int& y0,
                                         int& z0) const {
    tile_origin(t, ntx, ntz, x0, y0, z0);
  }
};

// Minimum lapse over the points of P's tile at (x0, y0, z0), read from
// global memory by one thread: the value tile_lapse_min takes from the
// centre block in the FP32 launch (the same points; fmin is exact, so the
// order does not matter).
__device__ __forceinline__ double tile_lapse_min_global(const Patch& P,
                                                        int x0, int y0,
                                                        int z0) {
  const int g = P.ghost;
  const int nx = P.n[0] - x0 < kLdsTile[0] ? P.n[0] - x0 : kLdsTile[0];
  const int ny = P.n[1] - y0 < kLdsTile[1] ? P.n[1] - y0 : kLdsTile[1];
  const int nz = P.n[2] - z0 < kLdsTile[2] ? P.n[2] - z0 : kLdsTile[2];
  const double* a = P.u_s + int64_t(ALP) * P.sf + int64_t(z0 + g) * P.sz +
                    int64_t(y0 + g) * P.sy + x0 + g;
  double m = 1.0e300;
  for (int dz = 0; dz < nz; ++dz)
    for (int dy = 0; dy < ny; ++dy) {
      const double* row = a + int64_t(dz) * P.sz + int64_t(dy) * P.sy;
      if (nx == kLdsTile[0]) {
#pragma unroll
        for (int dx = 0; dx < kLdsTile[0]; ++dx) m = fmin(m, row[dx]);
      } else {
        for (int dx = 0; dx < nx; ++dx) m = fmin(m, row[dx]);
      }
    }
  return m;
}

// Writes val of every thread whose flag is set to list, in thread order,
// and returns their number (the same in every thread).  wcnt: 4 ints of
// LDS.  Contains the barriers that make list readable afterwards.
__device__ __forceinline__ int compact_flags(bool f, int val, int* list,
                                             int* wcnt) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t mask = __builtin_amdgcn_ballot_w64(f);
  if (lane == 0) wcnt[wave] = __builtin_popcountll(mask);
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    base += w < wave ? wcnt[w] : 0;
    tot += wcnt[w];
  }
  const int below = __builtin_amdgcn_mbcnt_hi(
      uint32_t(mask >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(mask), 0));
  if (f) list[base + below] = val;
  __syncthreads();
  return tot;
}

// One patch, mixed precision, second launch: the FP64 tiles.  Workgroup b
// examines the tiles t = (i * perm) mod ntiles for i in its share of an
// even split of 0 .. ntiles - 1, one tile per thread at a time.  perm is
// coprime to ntiles, so every tile is examined exactly once, and the tiles
// around a puncture (neighbours in the numbering) land on many workgroups.
// The tiles whose minimum lapse is below the threshold run through the FP64
// pipeline.
template <int ORDER, bool KSH = false>
__global__ void __launch_bounds__(256)
    k_stage_lds_f64tiles(const Patch P, const Gauge G, const int stage,
                         const TileMap M, const int perm,
                         double* const kout) {
  using Geo = TileGeo<ORDER>;
  __shared__ __attribute__((aligned(16))) double ring[Geo::NBUF * Geo::BUFD];
  __shared__ __attribute__((aligned(16))) double sc[kNCentre * 256];
  __shared__ __attribute__((aligned(16))) double mixs[mix_doubles<Geo>()];
  __shared__ int list[256];
  // the 4 per-wave counts of compact_flags live in the mixed-derivative
  // scratch, which is idle between lds_tiles calls (the LDS is full)
  int* wcnt = (int*)mixs;
  const int tid = threadIdx.x;
  int lo, hi;
  walk_range(blockIdx.x, gridDim.x, M.ntiles, lo, hi);
  for (int c0 = lo; c0 < hi; c0 += 256) {
    bool f = false;
    int t = 0;
    if (c0 + tid < hi) {
      t = int((int64_t(c0 + tid) * perm) % M.ntiles);
      int x0, y0, z0;
      tile_origin(t, M.ntx, M.ntz, x0, y0, z0);
      f = tile_lapse_min_global(P, x0, y0, z0) < G.alpha_thr;
    }
    const int n = compact_flags(f, t, list, wcnt);
    if (n > 0) {
      const ListWalk w{(const lds_int*)list, n, M.ntx, M.ntz};
      lds_tiles<ORDER, TP_F64, true, TileGeo<ORDER>, ListWalk, KSH>(
          P, G, stage, w, ring, sc, mixs, kout);
    }
    __syncthreads();  // ring, sc, list and wcnt are reused
  }
}

// Many patches, FP64: workgroup b runs the items [wstart[q], wstart[q+1])
// for q = walk_pos(b).
template <int ORDER>
__global__ void __launch_bounds__(256)
    k_stage_lds_batch(const Patch* __restrict__ patches,
                      const LdsItem* __restrict__ items,
                      const int32_t* __restrict__ wstart, const Gauge G,
                      const int stage) {
  using Geo = TileGeo<ORDER>;
  __shared__ __attribute__((aligned(16))) double ring[Geo::NBUF * Geo::BUFD];
  __shared__ __attribute__((aligned(16))) double sc[kNCentre * 256];
  __shared__ __attribute__((aligned(16))) double mixs[mix_doubles<Geo>()];
  const int q = walk_pos(blockIdx.x, gridDim.x);
  const int i0 = wstart[q], i1 = wstart[q + 1];
  for (int i = i0; i < i1; ++i) {
    const LdsItem it = items[i];
    const Patch P = patches[it.patch];
    const Walk w = walk_contig(it.tlo, it.thi - it.tlo, it.ntx, it.ntz);
    // trimmed DMA always: many patches at once miss L2 more often, so the
    // saved traffic matters more than the register
    lds_tiles<ORDER, TP_F64, true>(P, G, stage, w, ring, sc, mixs);
    __builtin_amdgcn_s_barrier();  // every wave is done with ring and sc
  }
}

// Many patches, mixed precision, first launch: the FP32 tiles, with split
// (1 or 2) workgroups per work list position.  Workgroup b' stands for
// workgroup b of the list's launch of nwg on the same XCD (b' mod 8 = b mod
// 8) and runs part h of every item of b's list.
template <int ORDER>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(ORDER == 4 ? 2 : 1,
                                       ORDER == 4 ? 2 : 1)))
    k_stage_lds_batch_f32(const Patch* __restrict__ patches,
                          const LdsItem* __restrict__ items,
                          const int32_t* __restrict__ wstart, const Gauge G,
                          const int stage, const int nwg, const int split) {
  using Geo = GeoF32<ORDER>;
  __shared__ __attribute__((aligned(16))) double ring[Geo::NBUF * Geo::BUFD];
  __shared__ __attribute__((aligned(16))) double sc[kNCentre * 256];
  __shared__ __attribute__((aligned(16))) double mixs[mix_doubles<Geo>()];
  const int bp = blockIdx.x;
  const bool xcd = (nwg & 7) == 0;
  const int b = xcd ? 8 * ((bp >> 3) / split) + (bp & 7) : bp / split;
  const int h = xcd ? (bp >> 3) % split : bp % split;
  const int q = walk_pos(b, nwg);
  const int i0 = wstart[q], i1 = wstart[q + 1];
  for (int i = i0; i < i1; ++i) {
    const LdsItem it = items[i];
    const Patch P = patches[it.patch];
    const int n = it.thi - it.tlo;
    const int lo = it.tlo + n * h / split, hi = it.tlo + n * (h + 1) / split;
    const Walk w = walk_contig(lo, hi - lo, it.ntx, it.ntz);
    lds_tiles<ORDER, TP_F32, true, Geo>(P, G, stage, w, ring, sc, mixs);
    __builtin_amdgcn_s_barrier();  // every wave is done with ring and sc
  }
}

// Many patches, mixed precision, second launch: the FP64 tiles.  Workgroup
// b examines the candidates [lo, hi) of an even split of cand (every tile of
// the launch once, scattered by the plan), one per thread at a time, as
// k_stage_lds_f64tiles does.
template <int ORDER>
__global__ void __launch_bounds__(256)
    k_stage_lds_batch_f64tiles(const Patch* __restrict__ patches,
                               const TileRef* __restrict__ cand,
                               const int ncand, const Gauge G,
                               const int stage) {
  using Geo = TileGeo<ORDER>;
  __shared__ __attribute__((aligned(16))) double ring[Geo::NBUF * Geo::BUFD];
  __shared__ __attribute__((aligned(16))) double sc[kNCentre * 256];
  __shared__ __attribute__((aligned(16))) double mixs[mix_doubles<Geo>()];
  __shared__ int list[256];
  int* wcnt = (int*)mixs;  // idle between lds_tiles calls (the LDS is full)
  const int tid = threadIdx.x;
  int lo, hi;
  walk_range(blockIdx.x, gridDim.x, ncand, lo, hi);
  for (int c0 = lo; c0 < hi; c0 += 256) {
    bool f = false;
    if (c0 + tid < hi) {
      const TileRef r = cand[c0 + tid];
      const Patch& P = patches[r.patch];
      const int ntx = (P.n[0] + kLdsTile[0] - 1) / kLdsTile[0];
      const int ntz = (P.n[2] + kLdsTile[2] - 1) / kLdsTile[2];
      int x0, y0, z0;
      tile_origin(r.tile, ntx, ntz, x0, y0, z0);
      f = tile_lapse_min_global(P, x0, y0, z0) < G.alpha_thr;
    }
    const int n = compact_flags(f, c0 + tid, list, wcnt);
    for (int k = 0; k < n; ++k) {
      const TileRef r = cand[list[k]];
      const Patch P = patches[r.patch];
      const OneWalk w{r.tile, (P.n[0] + kLdsTile[0] - 1) / kLdsTile[0],
                      (P.n[2] + kLdsTile[2] - 1) / kLdsTile[2]};
      lds_tiles<ORDER, TP_F64, true>(P, G, stage, w, ring, sc, mixs);
      __syncthreads();  // every wave is done with ring and sc
    }
    __syncthreads();  // the lists and wcnt are reused
  }
}

template <int ORDER>
inline TileMap lds_tile_map(const Patch& P) {
  using Geo = TileGeo<ORDER>;
  TileMap M;
  M.ntx = (P.n[0] + Geo::TX - 1) / Geo::TX;
  M.nty = (P.n[1] + Geo::TY - 1) / Geo::TY;
  M.ntz = (P.n[2] + Geo::TZ - 1) / Geo::TZ;
  M.ntiles = M.ntx * M.nty * M.ntz;
  M.bx = M.by = M.bz = 0;
  return M;
}

// Blocked walk (Walk with bx > 0) for a launch of 256 or 512 workgroups
// (one or two per CU): the first block shape of nwg / 8 tiles that divides
// the tile grid and leaves every XCD at least one block; otherwise the
// contiguous walk.  Order 8 (a 14-plane box) measured best with blocks 2
// tiles deep in z, order 4 with 4.
template <int ORDER>
inline void choose_blocks(TileMap& M, int nwg) {
  static const int s32[][3] = {
      {4, ORDER == 8 ? 4 : 2, ORDER == 8 ? 2 : 4},
      {4, ORDER == 8 ? 2 : 4, ORDER == 8 ? 4 : 2},
      {2, 4, 4}, {2, 2, 8}, {4, 8, 1}, {8, 4, 1}};
  static const int s64[][3] = {{4, 4, 4}, {4, 8, 2}, {8, 4, 2},
                               {2, 8, 4}, {4, 2, 8}, {8, 8, 1}};
  M.bx = M.by = M.bz = 0;
  if (nwg != 256 && nwg != 512) return;
  for (const auto& b : (nwg == 256 ? s32 : s64)) {
    if (M.ntx % b[0] || M.nty % b[1] || M.ntz % b[2]) continue;
    if ((M.ntx / b[0]) * (M.nty / b[1]) < 8) continue;
    M.bx = b[0];
    M.by = b[1];
    M.bz = b[2];
    return;
  }
}

// The LDS path needs 16-byte aligned granules: (u + ghost - R - 1) aligned
// and even strides.
template <int ORDER>
inline bool lds_path_ok(const Patch& P) {
  using Geo = TileGeo<ORDER>;
  const uintptr_t a = reinterpret_cast<uintptr_t>(P.u_s) +
                      8u * uintptr_t(P.ghost - Geo::R - 1);
  return (a % 16) == 0 && (P.sy % 2) == 0 && (P.sz % 2) == 0 &&
         (P.sf % 2) == 0;
}

}  // namespace bssn

namespace bssn {

// precision 0: one FP64 launch.  Mixed: the FP32 tiles (two workgroups per
// CU at order 4), then the FP64 tiles; both launches take the same per-tile
// decision from the stage input, so each tile is written exactly once.
template <int ORDER, bool KSH>
hipError_t launch_stage_lds_k(const Patch& P, const Gauge& G, int stage,
                              int precision, int nwg_max, hipStream_t st,
                              double* kout) {
  TileMap M = lds_tile_map<ORDER>(P);
  const int nwg = M.ntiles < nwg_max ? M.ntiles : nwg_max;
  if (precision == 0) {
    choose_blocks<ORDER>(M, nwg);
    hipLaunchKernelGGL((k_stage_lds<ORDER, KSH>), dim3(nwg), dim3(256), 0, st,
                       P, G, stage, M, kout);
    return hipGetLastError();
  }
  const int per_cu = ORDER == 4 ? 2 : 1;
  const int nwg32 = M.ntiles < per_cu * nwg_max ? M.ntiles : per_cu * nwg_max;
  TileMap M32 = M;
  choose_blocks<ORDER>(M32, nwg32);
  hipLaunchKernelGGL((k_stage_lds_f32<ORDER, KSH>), dim3(nwg32), dim3(256), 0,
                     st, P, G, stage, M32, kout);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_stage_lds_f64tiles<ORDER, KSH>), dim3(nwg), dim3(256),
                     0, st, P, G, stage, M, int(tile_perm(M.ntiles)), kout);
  return hipGetLastError();
}
// kout set: the kernels that also store the right-hand side at the
// outermost interior layer there.
template <int ORDER>
hipError_t launch_stage_lds(const Patch& P, const Gauge& G, int stage,
                            int precision, int nwg_max, hipStream_t st,
                            double* kout = nullptr) {
  return kout ? launch_stage_lds_k<ORDER, true>(P, G, stage, precision,
                                                nwg_max, st, kout)
              : launch_stage_lds_k<ORDER, false>(P, G, stage, precision,
                                                 nwg_max, st, nullptr);
}

// Explicit-variant launch of one static patch, and batched launches.
template <int ORDER>
hipError_t launch_patch_t(const Patch& P, const Gauge& G, int stage,
                          int precision, int variant, int nwg,
                          hipStream_t st) {
  switch (variant) {
    case VAR_LDS:
      return launch_stage_lds<ORDER>(P, G, stage, precision, nwg, st);
    case VAR_D64:
    case VAR_D64Z4:  // per patch, one plane per workgroup (same results)
      return launch_stage_variant<ORDER, false>(P, G, stage, precision, 64,
                                                st);
    case VAR_D32:
    case VAR_D32Z4:
      return launch_stage_variant<ORDER, false>(P, G, stage, precision, 32,
                                                st);
  }
  return hipErrorInvalidValue;
}

template <int ORDER>
bool variant_ok_t(const Patch& P, int variant) {
  if (variant != VAR_LDS) return variant > VAR_LDS && variant < NVAR;
  Patch q = P;
  const double* bufs[4] = {P.u_s, P.u_n, P.acc, P.out};
  for (const double* b : bufs) {
    if (!b) continue;
    q.u_s = b;
    if (!lds_path_ok<ORDER>(q)) return false;
  }
  return true;
}

template <int ORDER>
hipError_t launch_batch_t(const BatchLaunch& B, const Gauge& G, int stage,
                          int precision, hipStream_t st) {
  if (B.variant == VAR_LDS) {
    const LdsItem* it = static_cast<const LdsItem*>(B.items);
    if (precision == 0) {
      hipLaunchKernelGGL((k_stage_lds_batch<ORDER>), dim3(B.nwg), dim3(256),
                         0, st, B.patches, it, B.wstart, G, stage);
      return hipGetLastError();
    }
    if (!B.cand) return hipErrorInvalidValue;  // the plan always builds it
    const int split = ORDER == 4 ? 2 : 1;
    hipLaunchKernelGGL((k_stage_lds_batch_f32<ORDER>), dim3(split * B.nwg),
                       dim3(256), 0, st, B.patches, it, B.wstart, G, stage,
                       B.nwg, split);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || B.ncand <= 0) return e;
    const int nwg64 = B.ncand < B.nwg ? B.ncand : B.nwg;
    hipLaunchKernelGGL((k_stage_lds_batch_f64tiles<ORDER>), dim3(nwg64),
                       dim3(256), 0, st, B.patches, B.cand, B.ncand, G,
                       stage);
    return hipGetLastError();
  }
  if (B.variant <= VAR_LDS || B.variant >= NVAR) return hipErrorInvalidValue;
  return launch_direct_batch<ORDER>(
      B.patches, static_cast<const DirectItem*>(B.items), B.nitems,
      kVarTile[B.variant][0], kVarTile[B.variant][2], G, stage, precision,
      st);
}

}  // namespace bssn
