// bssn_batch.cpp -- many independent static patches advanced together (the
// mesh-refinement picture of the paper's section on adaptive mesh
// refinement: each refinement level is a set of independent component
// grids of uneven sizes, all evolved with the same right-hand side).
//
// A plan sorts the patches into size classes (largest extent rounded up to
// a multiple of 16 points), picks one kernel variant per class (timed trial
// launches, or a default), and builds per variant a device work list over
// all patches of the classes that chose it:
//   VAR_LDS  runs of LDS tiles: one persistent workgroup per compute unit;
//            whole patches are assigned to XCDs (balanced by tile count) and
//            each patch's tiles are split evenly over the workgroups of its
//            XCD, one item (patch, first tile, end tile) per workgroup;
//            in mixed precision two workgroups per compute unit share each
//            item's tiles (FP32 tiles), then an FP64 pass examines every
//            tile of the list's patches (candidate list in scattered order);
//   VAR_D*   one item per direct-kernel workgroup (patch, x0, y0, z0): a
//            64 x 4 or 32 x 8 tile of one plane or of a 4-plane z-block.
// The four stages of an RK4 step (one launch per variant in use per stage)
// are captured once into a hipGraph; batch_patches replays it per step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/bssn.h"
#include "bssn_api_internal.h"
#include "bssn_internal.h"
#include "bssn_kernels.h"

namespace bssn {
namespace {

constexpr int kMaxPatches = 1 << 16;
constexpr int kTuneReps = 3;

int class_extent(const bssn_grid& g) {
  const int m = std::max(g.n[0], std::max(g.n[1], g.n[2]));
  return (m + 15) / 16 * 16;
}

// Tile counts of patch g for the LDS kernel.
void lds_tiles_of(const bssn_grid& g, int& ntx, int& nty, int& ntz) {
  ntx = (g.n[0] + kLdsTile[0] - 1) / kLdsTile[0];
  nty = (g.n[1] + kLdsTile[1] - 1) / kLdsTile[1];
  ntz = (g.n[2] + kLdsTile[2] - 1) / kLdsTile[2];
}

// Host work list of one variant over a list of patches.
struct HostGroup {
  int variant = VAR_LDS;
  int nwg = 0;                      // VAR_LDS workgroups
  std::vector<LdsItem> lds;         // VAR_LDS items
  std::vector<int32_t> wstart;      // VAR_LDS, nwg + 1
  std::vector<DirectItem> direct;   // VAR_D*
  std::vector<TileRef> cand;        // VAR_LDS, mixed: FP64-pass candidates
  size_t item_bytes() const {
    return variant == VAR_LDS ? lds.size() * sizeof(LdsItem)
                              : direct.size() * sizeof(DirectItem);
  }
  int nitems() const {
    return int(variant == VAR_LDS ? lds.size() : direct.size());
  }
};

// Every LDS tile of the patches pids once, in the scattering order
// i -> (i * tile_perm(T)) mod T of their joint numbering (patches in list
// order, tiles in TileMap order), so that an even split of the list puts
// the tiles around a puncture on many workgroups of the FP64 pass.
int build_candidates(const std::vector<bssn_grid>& grids,
                     const std::vector<int>& pids, HostGroup& G) {
  std::vector<int64_t> base(pids.size() + 1, 0);
  for (size_t i = 0; i < pids.size(); ++i) {
    int ntx, nty, ntz;
    lds_tiles_of(grids[pids[i]], ntx, nty, ntz);
    base[i + 1] = base[i] + int64_t(ntx) * nty * ntz;
  }
  const int64_t T = base.back();
  if (T >= (int64_t(1) << 31))
    return fail(BSSN_EUNSUPPORTED, "batch: %lld LDS tiles exceed the "
                "candidate list range", (long long)T);
  const int64_t perm = tile_perm(T);
  G.cand.resize(size_t(T));
  for (int64_t i = 0; i < T; ++i) {
    const int64_t t = (i * perm) % T;
    const size_t j =
        size_t(std::upper_bound(base.begin(), base.end(), t) - base.begin()) -
        1;
    G.cand[size_t(i)] = TileRef{pids[j], int32_t(t - base[j])};
  }
  return BSSN_OK;
}

// mixed: also the FP64-pass candidates of a VAR_LDS group.
int build_group(const std::vector<bssn_grid>& grids,
                const std::vector<int>& pids, int variant, int nwg_max,
                bool mixed, HostGroup& G) {
  G = HostGroup();
  G.variant = variant;
  if (variant == VAR_LDS) {
    if (mixed) {
      const int rc = build_candidates(grids, pids, G);
      if (rc) return rc;
    }
    // XCD-affine: workgroup b runs on XCD b mod 8 and takes the item list
    // of position q = walk_pos(b), so positions [x*W, (x+1)*W) (W = nwg/8)
    // are the workgroups of XCD x.  Whole patches go to XCDs by a
    // longest-processing-time greedy on tile count; each patch's tiles are
    // split evenly over its XCD's W workgroups, in the single-patch order,
    // so neighbouring columns run at the same time on one XCD and their
    // halos meet in its L2, and a workgroup's share of a patch (tiles / W)
    // is long compared with the drift between workgroups.  Patches smaller
    // than W tiles start at a rotating offset.  With nwg not a multiple
    // of 8 the whole GPU acts as one group.
    std::vector<int64_t> tiles(pids.size());
    int64_t T = 0;
    for (size_t i = 0; i < pids.size(); ++i) {
      int ntx, nty, ntz;
      lds_tiles_of(grids[pids[i]], ntx, nty, ntz);
      tiles[i] = int64_t(ntx) * nty * ntz;
      T += tiles[i];
      if (tiles[i] >= (int64_t(1) << 31) / 2)
        return fail(BSSN_EUNSUPPORTED, "batch: a patch of %lld LDS tiles "
                    "exceeds the work-list range", (long long)tiles[i]);
    }
    const int nwg = int(std::min<int64_t>(nwg_max, T));
    const int ngrp = (nwg % 8 == 0) ? 8 : 1;
    const int W = nwg / ngrp;
    G.nwg = nwg;
    // A patch larger than one group's fair share (T / ngrp) is spread over
    // every group: group x takes the x-th eighth of its tiles.  Smaller
    // patches go whole to the least-loaded group, largest first.
    struct Piece {
      int i;
      int64_t lo, hi;
    };
    std::vector<std::vector<Piece>> mine(ngrp);
    std::vector<int64_t> load(ngrp, 0);
    std::vector<int> order(pids.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = int(i);
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return tiles[x] > tiles[y]; });
    for (int i : order) {
      if (ngrp > 1 && tiles[i] * ngrp >= T) {
        for (int x = 0; x < ngrp; ++x) {
          const Piece pc{i, tiles[i] * x / ngrp, tiles[i] * (x + 1) / ngrp};
          load[x] += pc.hi - pc.lo;
          mine[x].push_back(pc);
        }
        continue;
      }
      const int x = int(std::min_element(load.begin(), load.end()) -
                        load.begin());
      load[x] += tiles[i];
      mine[x].push_back(Piece{i, 0, tiles[i]});
    }
    std::vector<std::vector<LdsItem>> per(nwg);
    for (int x = 0; x < ngrp; ++x) {
      std::sort(mine[x].begin(), mine[x].end(),
                [](const Piece& a, const Piece& b) { return a.i < b.i; });
      int rot = 0;
      for (const Piece& pc : mine[x]) {
        LdsItem it;
        it.patch = pids[pc.i];
        lds_tiles_of(grids[pids[pc.i]], it.ntx, it.nty, it.ntz);
        const int64_t t = pc.hi - pc.lo;
        for (int l = 0; l < W; ++l) {
          const int64_t lo = pc.lo + t * l / W, hi = pc.lo + t * (l + 1) / W;
          if (hi <= lo) continue;
          it.tlo = int32_t(lo);
          it.thi = int32_t(hi);
          per[x * W + (t < W ? (l + rot) % W : l)].push_back(it);
        }
        if (t < W) rot = int((rot + t) % W);
      }
    }
    G.wstart.assign(nwg + 1, 0);
    for (int q = 0; q < nwg; ++q) {
      G.wstart[q] = int32_t(G.lds.size());
      G.lds.insert(G.lds.end(), per[q].begin(), per[q].end());
    }
    if (G.lds.size() >= size_t(1) << 31)
      return fail(BSSN_EUNSUPPORTED, "batch: work list too long");
    G.wstart[nwg] = int32_t(G.lds.size());
    return BSSN_OK;
  }
  const int bx = kVarTile[variant][0], by = kVarTile[variant][1];
  const int bz = kVarTile[variant][2];
  int64_t count = 0;
  for (int p : pids) {
    const bssn_grid& g = grids[p];
    count += int64_t((g.n[0] + bx - 1) / bx) * ((g.n[1] + by - 1) / by) *
             ((g.n[2] + bz - 1) / bz);
  }
  if (count >= (int64_t(1) << 31) - 1)
    return fail(BSSN_EUNSUPPORTED, "batch: %lld workgroups exceed one launch",
                (long long)count);
  G.direct.reserve(size_t(count));
  for (int p : pids) {
    const bssn_grid& g = grids[p];
    for (int z0 = 0; z0 < g.n[2]; z0 += bz)
      for (int y0 = 0; y0 < g.n[1]; y0 += by)
        for (int x0 = 0; x0 < g.n[0]; x0 += bx)
          G.direct.push_back(DirectItem{p, x0, y0, z0});
  }
  return BSSN_OK;
}

size_t align256(size_t n) { return (n + 255) / 256 * 256; }

// Device copy of a group's work list (items, then wstart) at dst.
// Device copy of a group's work list (items, wstart, then the candidates)
// at dst.
size_t group_bytes(const HostGroup& G) {
  return align256(G.item_bytes()) + align256(G.wstart.size() * 4) +
         align256(G.cand.size() * sizeof(TileRef));
}
hipError_t upload_group(const HostGroup& G, char* dst, BatchLaunch& L) {
  L.variant = G.variant;
  L.items = dst;
  L.nitems = G.nitems();
  L.nwg = G.nwg;
  L.wstart = nullptr;
  L.cand = nullptr;
  L.ncand = 0;
  const void* src = G.variant == VAR_LDS ? (const void*)G.lds.data()
                                         : (const void*)G.direct.data();
  hipError_t e = hipMemcpy(dst, src, G.item_bytes(), hipMemcpyHostToDevice);
  if (e != hipSuccess || G.variant != VAR_LDS) return e;
  char* w = dst + align256(G.item_bytes());
  L.wstart = reinterpret_cast<const int32_t*>(w);
  e = hipMemcpy(w, G.wstart.data(), G.wstart.size() * 4,
                hipMemcpyHostToDevice);
  if (e != hipSuccess || G.cand.empty()) return e;
  char* c = w + align256(G.wstart.size() * 4);
  L.cand = reinterpret_cast<const TileRef*>(c);
  L.ncand = int(G.cand.size());
  return hipMemcpy(c, G.cand.data(), G.cand.size() * sizeof(TileRef),
                   hipMemcpyHostToDevice);
}

struct AddrRange {
  hipDeviceptr_t base;
  size_t size;
};

}  // namespace
}  // namespace bssn

using namespace bssn;

struct bssn_batch_plan {
  int device = -1;
  int order = 4, precision = 0, np = 0;
  Gauge G{};
  std::vector<bssn_grid> grids;
  std::vector<Patch> hp[4];           // per stage, per patch
  std::vector<const void*> ptrs;      // every buffer the plan touches
  std::vector<AddrRange> ranges;      // their allocations at plan time
  struct Cls {
    int extent, variant;
    float ms[NVAR];
    std::vector<int> pids;
  };
  std::vector<Cls> classes;
  std::vector<int> var_of_patch;
  char* dmem = nullptr;               // Patch[4][np], then work lists
  std::vector<BatchLaunch> launches;  // one per variant in use (stage-free)
  int mode = 0;                       // kPersistent or kPerPatch
  float mode_ms[2] = {-1.f, -1.f};    // tuned stage-0 times per mode
  hipStream_t cs = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraph_t sgraph[4] = {};          // one stage each (batch_patches_stage)
  hipGraphExec_t sexec[4] = {};

  ~bssn_batch_plan() {
    for (int s = 0; s < 4; ++s) {
      if (sexec[s]) (void)hipGraphExecDestroy(sexec[s]);
      if (sgraph[s]) (void)hipGraphDestroy(sgraph[s]);
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cs) (void)hipStreamDestroy(cs);
    if (dmem) (void)hipFree(dmem);
  }
  const Patch* dpatches(int stage) const {
    return reinterpret_cast<const Patch*>(dmem) + size_t(stage) * np;
  }
};

namespace bssn {
namespace {

// Records the allocation of every buffer; returns BSSN_ESTALE when one of
// them is no longer the allocation it was at plan time.
int check_fresh(const bssn_batch_plan* plan) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != plan->device)
    return fail(BSSN_ESTALE, "batch plan belongs to device %d, current is %d",
                plan->device, dev);
  for (size_t i = 0; i < plan->ptrs.size(); ++i) {
    AddrRange r{};
    e = hipMemGetAddressRange(&r.base, &r.size,
                              (hipDeviceptr_t)plan->ptrs[i]);
    if (e != hipSuccess) {
      (void)hipGetLastError();  // do not leave the query's error behind
      return fail(BSSN_ESTALE, "batch plan buffer %zu (patch %zu) is no "
                  "longer allocated", i % 5, i / 5);
    }
    if (r.base != plan->ranges[i].base || r.size != plan->ranges[i].size)
      return fail(BSSN_ESTALE, "batch plan buffer %zu (patch %zu) lies in a "
                  "different allocation than at plan time", i % 5, i / 5);
  }
  return BSSN_OK;
}

// Launch modes of a plan's graph: the persistent work-list kernels (one
// launch per tile in use per stage), or one launch per patch and stage
// (the same kernels batch_patches_unbatched uses).
enum : int { kPersistent = 0, kPerPatch = 1 };

hipError_t enqueue_stages(bssn_batch_plan* P, int mode, int s0, int s1,
                          hipStream_t st) {
  const int nwg = persistent_groups();
  for (int s = s0; s < s1; ++s) {
    if (mode == kPersistent) {
      for (BatchLaunch L : P->launches) {
        L.patches = P->dpatches(s);
        hipError_t e = launch_batch(L, P->G, P->order, s, P->precision, st);
        if (e != hipSuccess) return e;
      }
    } else {
      for (int p = 0; p < P->np; ++p) {
        hipError_t e = launch_patch(P->hp[s][p], P->G, P->order, s,
                                    P->precision, P->var_of_patch[p], nwg, st);
        if (e != hipSuccess) return e;
      }
    }
  }
  return hipSuccess;
}

// Captures stages [s0, s1) in `mode` on the plan's private stream.
int capture(bssn_batch_plan* P, int mode, int s0, int s1, hipGraph_t* g,
            hipGraphExec_t* x) {
  *g = nullptr;
  *x = nullptr;
  hipError_t e = hipStreamBeginCapture(P->cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  const hipError_t le = enqueue_stages(P, mode, s0, s1, P->cs);
  e = hipStreamEndCapture(P->cs, g);
  if (le != hipSuccess) {
    if (*g) (void)hipGraphDestroy(*g);
    *g = nullptr;
    return hip_fail(le, "batch stage capture");
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(x, *g, nullptr, nullptr, 0);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  return BSSN_OK;
}

// Milliseconds of one replay of a stage-0 graph of `mode` (best of
// kTuneReps after a warm-up), or < 0 with *rc set on failure.
float time_mode(bssn_batch_plan* P, int mode, hipStream_t st, int* rc) {
  hipGraph_t g = nullptr;
  hipGraphExec_t x = nullptr;
  if ((*rc = capture(P, mode, 0, 1, &g, &x))) return -1.f;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float best = -1.f;
  for (int r = 0; r <= kTuneReps && e == hipSuccess; ++r) {
    e = hipEventRecord(e0, st);
    if (e == hipSuccess) e = hipGraphLaunch(x, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && r > 0 && (best < 0.f || ms < best)) best = ms;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipGraphExecDestroy(x);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    *rc = hip_fail(e, "launch-mode timing");
    return -1.f;
  }
  *rc = BSSN_OK;
  return best;
}

// The step graph: launch mode (timed when tuning), then stages 0..3.
int record_graph(bssn_batch_plan* P, int autotune, hipStream_t st) {
  hipError_t e = hipStreamCreateWithFlags(&P->cs, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
  P->mode = (autotune & BSSN_BATCH_PER_PATCH) ? kPerPatch : kPersistent;
  if (autotune == 1) {
    for (int m = 0; m < 2; ++m) {
      int rc = BSSN_OK;
      P->mode_ms[m] = time_mode(P, m, st, &rc);
      if (rc) return rc;
    }
    P->mode = P->mode_ms[kPerPatch] < P->mode_ms[kPersistent] ? kPerPatch
                                                              : kPersistent;
  }
  int rc = capture(P, P->mode, 0, 4, &P->graph, &P->exec);
  for (int s = 0; s < 4 && rc == BSSN_OK; ++s)
    rc = capture(P, P->mode, s, s + 1, &P->sgraph[s], &P->sexec[s]);
  return rc;
}

// Milliseconds of one batched stage-0 launch of variant v over pids (best
// of kTuneReps after one warm-up), or < 0 on failure.
float time_variant(bssn_batch_plan* P, const std::vector<int>& pids, int v,
                   hipStream_t st, int* rc) {
  HostGroup H;
  if ((*rc = build_group(P->grids, pids, v, persistent_groups(),
                         P->precision != 0, H)))
    return -1.f;
  char* d = nullptr;
  hipError_t e = hipMalloc((void**)&d, group_bytes(H));
  if (e != hipSuccess) {
    *rc = fail(BSSN_ENOMEM, "autotune work list: %s", hipGetErrorString(e));
    return -1.f;
  }
  BatchLaunch L{};
  e = upload_group(H, d, L);
  L.patches = P->dpatches(0);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float best = -1.f;
  for (int r = 0; r <= kTuneReps && e == hipSuccess; ++r) {
    e = hipEventRecord(e0, st);
    if (e == hipSuccess) e = launch_batch(L, P->G, P->order, 0, P->precision, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && r > 0 && (best < 0.f || ms < best)) best = ms;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(d);
  if (e != hipSuccess) {
    *rc = hip_fail(e, "autotune launch");
    return -1.f;
  }
  *rc = BSSN_OK;
  return best;
}

int plan_build(bssn_batch_plan* P, int autotune, hipStream_t st) {
  const int np = P->np;
  // size classes, in increasing extent
  std::vector<int> ext(np);
  for (int p = 0; p < np; ++p) ext[p] = class_extent(P->grids[p]);
  std::vector<int> order(np);
  for (int p = 0; p < np; ++p) order[p] = p;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return ext[a] < ext[b]; });
  for (int p : order) {
    if (P->classes.empty() || P->classes.back().extent != ext[p]) {
      bssn_batch_plan::Cls c;
      c.extent = ext[p];
      c.variant = -1;
      for (float& m : c.ms) m = -1.f;
      P->classes.push_back(c);
    }
    P->classes.back().pids.push_back(p);
  }
  // device patch records
  const size_t pbytes = align256(sizeof(Patch) * 4 * size_t(np));
  // variants a class may use
  P->var_of_patch.assign(np, VAR_LDS);
  for (auto& c : P->classes) {
    bool lds_ok = true;
    for (int p : c.pids)
      for (int s = 0; s < 4; ++s)
        lds_ok = lds_ok && variant_ok(P->hp[s][p], P->order, VAR_LDS);
    const int dflt = lds_ok ? VAR_LDS : (c.extent > 32 ? VAR_D64 : VAR_D32);
    c.variant = dflt;
    if (autotune & 0x100) {
      c.variant = autotune & 0xff;
      if (c.variant == VAR_LDS && !lds_ok)
        return fail(BSSN_EINVAL, "forced LDS tile: a patch of class %d has "
                    "buffers the LDS kernel cannot address in 16-byte "
                    "granules", c.extent);
    } else if (autotune == 1) {
      // patch records must be on the device for the trial launches
      if (!P->dmem) {
        hipError_t e = hipMalloc((void**)&P->dmem, pbytes);
        if (e != hipSuccess)
          return fail(BSSN_ENOMEM, "batch patches: %s", hipGetErrorString(e));
        for (int s = 0; s < 4; ++s) {
          e = hipMemcpy(P->dmem + sizeof(Patch) * size_t(s) * np,
                        P->hp[s].data(), sizeof(Patch) * np,
                        hipMemcpyHostToDevice);
          if (e != hipSuccess) return hip_fail(e, "batch patch upload");
        }
      }
      float best = -1.f;
      for (int v = 0; v < NVAR; ++v) {
        if (v == VAR_LDS && !lds_ok) continue;
        int rc = BSSN_OK;
        const float ms = time_variant(P, c.pids, v, st, &rc);
        if (rc) return rc;
        c.ms[v] = ms;
        if (ms >= 0.f && (best < 0.f || ms < best)) {
          best = ms;
          c.variant = v;
        }
      }
    }
    for (int p : c.pids) P->var_of_patch[p] = c.variant;
  }
  // one work list per variant in use, patches in class order
  std::vector<HostGroup> groups;
  for (int v = 0; v < NVAR; ++v) {
    std::vector<int> pids;
    for (auto& c : P->classes)
      if (c.variant == v) pids.insert(pids.end(), c.pids.begin(), c.pids.end());
    if (pids.empty()) continue;
    groups.emplace_back();
    int rc = build_group(P->grids, pids, v, persistent_groups(),
                         P->precision != 0, groups.back());
    if (rc) return rc;
  }
  size_t total = pbytes;
  for (auto& g : groups) total += group_bytes(g);
  if (P->dmem) {
    (void)hipFree(P->dmem);
    P->dmem = nullptr;
  }
  hipError_t e = hipMalloc((void**)&P->dmem, total);
  if (e != hipSuccess)
    return fail(BSSN_ENOMEM, "batch work lists (%zu bytes): %s", total,
                hipGetErrorString(e));
  for (int s = 0; s < 4; ++s) {
    e = hipMemcpy(P->dmem + sizeof(Patch) * size_t(s) * np, P->hp[s].data(),
                  sizeof(Patch) * np, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "batch patch upload");
  }
  char* cur = P->dmem + pbytes;
  for (auto& g : groups) {
    BatchLaunch L{};
    e = upload_group(g, cur, L);
    if (e != hipSuccess) return hip_fail(e, "batch work-list upload");
    P->launches.push_back(L);
    cur += group_bytes(g);
  }
  return record_graph(P, autotune, st);
}

}  // namespace
}  // namespace bssn

extern "C" {

namespace {
// batch_patches_plan with stage 3 writing u_new[p] (NULL: u[p] itself).
int plan_create(int npatch, const bssn_grid* grids, const bssn_params* params,
                double* const* u, double* const* u_new, double* const* a,
                double* const* b, double* const* acc, const double* dt,
                int autotune, bssn_batch_plan** plan, void* stream) {
  if (!plan) return fail(BSSN_EINVAL, "plan is NULL");
  *plan = nullptr;
  int rc = check_params(params);
  if (rc) return rc;
  if (npatch < 1 || npatch > kMaxPatches)
    return fail(BSSN_EINVAL, "npatch = %d outside 1..%d", npatch, kMaxPatches);
  if (!grids || !u || !a || !b || !acc || !dt)
    return fail(BSSN_EINVAL, "grids, dt and the buffer arrays must be "
                "non-NULL");
  for (int p = 0; p < npatch; ++p)
    if (!std::isfinite(dt[p]) || dt[p] < 0.0)
      return fail(BSSN_EINVAL, "patch %d: dt = %g is not a finite value "
                  ">= 0", p, dt[p]);
  {
    const int flags = autotune & ~0xff, v = autotune & 0xff;
    const bool ok =
        autotune == 0 || autotune == 1 ||
        ((flags & ~(0x100 | BSSN_BATCH_PER_PATCH)) == 0 && flags != 0 &&
         ((flags & 0x100) ? v < NVAR : v == 0));
    if (!ok)
      return fail(BSSN_EINVAL, "autotune = %d: 0, 1, BSSN_BATCH_TILE(0..%d) "
                  "and/or BSSN_BATCH_PER_PATCH", autotune, NVAR - 1);
  }
  for (int p = 0; p < npatch; ++p) {
    if ((rc = check_grid(&grids[p], params->fd_order)))
      return fail(rc, "patch %d: %s", p, bssn_last_error());
    if (grids[p].bc != BSSN_BC_STATIC)
      return fail(BSSN_EINVAL, "patch %d: batched patches need "
                  "BSSN_BC_STATIC", p);
    const double* q[4] = {u[p], a[p], b[p], acc[p]};
    for (int i = 0; i < 4; ++i) {
      if (!q[i]) return fail(BSSN_EINVAL, "patch %d: buffer %d is NULL", p, i);
      for (int j = 0; j < i; ++j)
        if (q[i] == q[j])
          return fail(BSSN_EINVAL, "patch %d: buffers %d and %d alias", p, j, i);
    }
    if (u_new) {
      if (!u_new[p]) return fail(BSSN_EINVAL, "patch %d: u_new is NULL", p);
      for (int j = 1; j < 4; ++j)
        if (u_new[p] == q[j])
          return fail(BSSN_EINVAL, "patch %d: u_new aliases buffer %d", p, j);
    }
  }
  bssn_batch_plan* P = new (std::nothrow) bssn_batch_plan();
  if (!P) return fail(BSSN_ENOMEM, "batch plan");
  hipError_t e = hipGetDevice(&P->device);
  if (e != hipSuccess) {
    delete P;
    return hip_fail(e, "hipGetDevice");
  }
  P->order = params->fd_order;
  P->precision = params->precision;
  P->np = npatch;
  P->G = make_gauge(params);
  P->grids.assign(grids, grids + npatch);
  // stage s reads u_s, writes out (rk4_stage semantics): u -> a -> b -> a -> u
  for (int s = 0; s < 4; ++s) P->hp[s].resize(npatch);
  for (int p = 0; p < npatch; ++p) {
    Patch base = make_patch(&grids[p]);
    base.dt = dt[p];
    base.u_n = u[p];
    base.acc = acc[p];
    const double* us[4] = {u[p], a[p], b[p], a[p]};
    double* out[4] = {a[p], b[p], a[p], u_new ? u_new[p] : u[p]};
    for (int s = 0; s < 4; ++s) {
      Patch q = base;
      q.u_s = us[s];
      q.out = out[s];
      P->hp[s][p] = q;
    }
    const void* bufs[5] = {u[p], a[p], b[p], acc[p],
                           u_new ? u_new[p] : u[p]};
    for (const void* ptr : bufs) {
      AddrRange r{};
      e = hipMemGetAddressRange(&r.base, &r.size, (hipDeviceptr_t)ptr);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        delete P;
        return fail(BSSN_EINVAL, "patch %d: a buffer is not device memory "
                    "of this device", p);
      }
      // every slot of the state must lie inside the buffer's allocation
      const uint64_t need = uint64_t(base.sf) * NSLOT * 8u;
      const uint64_t beg = reinterpret_cast<uint64_t>(ptr);
      const uint64_t lo = reinterpret_cast<uint64_t>(r.base);
      if (beg < lo || beg - lo + need > uint64_t(r.size)) {
        delete P;
        return fail(BSSN_EINVAL, "patch %d: a buffer's allocation ends "
                    "before the %d slots of its grid", p, NSLOT);
      }
      P->ptrs.push_back(ptr);
      P->ranges.push_back(r);
    }
  }
  rc = plan_build(P, autotune, (hipStream_t)stream);
  if (rc) {
    delete P;
    return rc;
  }
  *plan = P;
  return BSSN_OK;
}
}  // namespace

int batch_patches_plan(int npatch, const bssn_grid* grids,
                       const bssn_params* params, double* const* u,
                       double* const* a, double* const* b,
                       double* const* acc, const double* dt, int autotune,
                       bssn_batch_plan** plan, void* stream) {
  return plan_create(npatch, grids, params, u, nullptr, a, b, acc, dt,
                     autotune, plan, stream);
}

int batch_patches_plan_out(int npatch, const bssn_grid* grids,
                           const bssn_params* params, double* const* u,
                           double* const* u_new, double* const* a,
                           double* const* b, double* const* acc,
                           const double* dt, int autotune,
                           bssn_batch_plan** plan, void* stream) {
  if (!u_new) {
    if (plan) *plan = nullptr;
    return fail(BSSN_EINVAL, "u_new is NULL");
  }
  return plan_create(npatch, grids, params, u, u_new, a, b, acc, dt,
                     autotune, plan, stream);
}

int batch_patches_stage(bssn_batch_plan* plan, int stage, void* stream) {
  if (!plan) return fail(BSSN_EINVAL, "plan is NULL");
  if (stage < 0 || stage > 3)
    return fail(BSSN_EINVAL, "stage = %d outside 0..3", stage);
  int rc = check_fresh(plan);
  if (rc) return rc;
  hipError_t e = hipGraphLaunch(plan->sexec[stage], (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch (stage)");
  return BSSN_OK;
}

int batch_patches(bssn_batch_plan* plan, int nsteps, void* stream) {
  if (!plan) return fail(BSSN_EINVAL, "plan is NULL");
  if (nsteps < 0) return fail(BSSN_EINVAL, "nsteps = %d < 0", nsteps);
  int rc = check_fresh(plan);
  if (rc) return rc;
  for (int k = 0; k < nsteps; ++k) {
    hipError_t e = hipGraphLaunch(plan->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  }
  return BSSN_OK;
}

int batch_patches_unbatched(bssn_batch_plan* plan, int nsteps, void* stream) {
  if (!plan) return fail(BSSN_EINVAL, "plan is NULL");
  if (nsteps < 0) return fail(BSSN_EINVAL, "nsteps = %d < 0", nsteps);
  int rc = check_fresh(plan);
  if (rc) return rc;
  const int nwg = persistent_groups();
  for (int k = 0; k < nsteps; ++k)
    for (int s = 0; s < 4; ++s)
      for (int p = 0; p < plan->np; ++p) {
        hipError_t e = launch_patch(plan->hp[s][p], plan->G, plan->order, s,
                                    plan->precision, plan->var_of_patch[p],
                                    nwg, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "per-patch stage launch");
      }
  return BSSN_OK;
}

int batch_patches_describe(const bssn_batch_plan* plan, int max_classes,
                           int32_t* out) {
  if (!plan) return fail(BSSN_EINVAL, "plan is NULL");
  if (max_classes < 0 || (max_classes > 0 && !out))
    return fail(BSSN_EINVAL, "out must hold 4 * max_classes entries");
  const int n = int(plan->classes.size());
  for (int i = 0; i < n && i < max_classes; ++i) {
    const auto& c = plan->classes[i];
    out[4 * i] = c.extent;
    for (int a = 0; a < 3; ++a) out[4 * i + 1 + a] = kVarTile[c.variant][a];
  }
  return n;
}

int batch_patches_launch_mode(const bssn_batch_plan* plan) {
  if (!plan) return fail(BSSN_EINVAL, "plan is NULL");
  return plan->mode == kPerPatch ? BSSN_BATCH_PER_PATCH : 0;
}

int batch_patches_destroy(bssn_batch_plan* plan) {
  delete plan;
  return BSSN_OK;
}

}  // extern "C"
