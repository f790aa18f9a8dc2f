// bssn_amr_plan.cpp -- the refinement-hierarchy plan (bssn_amr_plan_*): the
// lattice of every level, the source of every ghost point of a refined
// patch, the coarse points that restriction overwrites, all as flat op
// lists on the device; and the fill / restrict entry points.
//
// Level L has spacing h_L = h_0 / 2^L and a lattice o_L + G h_L (G integer
// per axis, o_L the origin of the level's first patch).  A refined level's
// points sit a quarter coarse spacing from coarse points:
// (o_L - o_{L-1}) / h_{L-1} = D - 1/4 with D integer.  In coarse index
// units a fine point G is at s = (q - 1/2)/2 with q = 2D + G, so the
// interpolation block starts at floor(s) - 1 = floor((q - 1)/2) - 1 and the
// point lies at 1.25 (q odd) or 1.75 (q even) of its nodes.  A coarse point
// G_c has its lower child at fine index 2(G_c - D).
#include <hip/hip_runtime.h>

#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "../../include/bssn.h"
#include "bssn_api_internal.h"
#include "bssn_kernels.h"

struct bssn_amr_plan {
  int npatch = 0, nlevel = 0, device = 0;
  std::vector<int64_t> fill_begin, fill_count;          // copy ops, per level
  std::vector<int64_t> tile_begin, tile_count, nprolong; // per level
  std::vector<int64_t> restr_begin, restr_count;        // per fine level
  bssn::AmrOp* d_ops = nullptr;
  bssn::AmrTile* d_tiles = nullptr;
  bssn::AmrGeo* d_geo = nullptr;
};

namespace bssn {
namespace {

int64_t floordiv(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

bool near_int(double x, int64_t* k) {
  const double r = std::nearbyint(x);
  if (!(std::fabs(x - r) <= 1e-6) || std::fabs(r) > 1e12) return false;
  *k = int64_t(r);
  return true;
}

struct Lat {          // one patch on its level's lattice
  int level;
  int64_t off[3];     // lattice index of interior point 0
  int n[3], g;
  int64_t st[3];      // element strides x, y, z
};

int64_t storage(const Lat& p, const int64_t idx[3]) {
  return idx[0] * p.st[0] + idx[1] * p.st[1] + idx[2] * p.st[2];
}

// Prolonged points of one 8 x 8 x 8 box of a fine patch that read one
// coarse patch: membership and the range of their block bases.
struct TileAcc {
  uint64_t mask[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int64_t bmin[3] = {INT64_MAX, INT64_MAX, INT64_MAX};
  int64_t bmax[3] = {INT64_MIN, INT64_MIN, INT64_MIN};
  int lo[3] = {8, 8, 8}, hi[3] = {-1, -1, -1};  // filled points in the box
};

}  // namespace
}  // namespace bssn

using namespace bssn;

extern "C" {

int bssn_amr_plan_create(const bssn_amr_patch* patches, int npatch,
                         bssn_amr_plan** out) {
  if (!out) return fail(BSSN_EINVAL, "out is NULL");
  *out = nullptr;
  if (!patches) return fail(BSSN_EINVAL, "patches is NULL");
  if (npatch < 1 || npatch > 65536)
    return fail(BSSN_EINVAL, "npatch = %d outside 1..65536", npatch);
  int nlevel = 0;
  for (int p = 0; p < npatch; ++p) {
    const bssn_amr_patch& P = patches[p];
    int rc = check_grid(&P.grid, 4);
    if (rc) return fail(rc, "patch %d: %s", p, bssn_last_error());
    if (P.grid.bc != BSSN_BC_STATIC)
      return fail(BSSN_EINVAL, "patch %d: bc must be BSSN_BC_STATIC", p);
    if (P.level < 0 || P.level > 30)
      return fail(BSSN_EINVAL, "patch %d: level %d outside 0..30", p,
                  P.level);
    if (P.level + 1 > nlevel) nlevel = P.level + 1;
  }
  // each level: its first patch sets the lattice
  std::vector<int> first(nlevel, -1);
  for (int p = 0; p < npatch; ++p)
    if (first[patches[p].level] < 0) first[patches[p].level] = p;
  for (int L = 0; L < nlevel; ++L)
    if (first[L] < 0) return fail(BSSN_EINVAL, "level %d has no patch", L);
  std::vector<int64_t> D(3 * nlevel, 0);
  for (int L = 1; L < nlevel; ++L) {
    const bssn_grid& f = patches[first[L]].grid;
    const bssn_grid& c = patches[first[L - 1]].grid;
    for (int a = 0; a < 3; ++a) {
      if (std::fabs(f.h[a] * 2.0 - c.h[a]) > 1e-12 * c.h[a])
        return fail(BSSN_EINVAL, "level %d: h[%d] is not half of level %d's",
                    L, a, L - 1);
      if (!near_int((f.origin[a] - c.origin[a]) / c.h[a] + 0.25,
                    &D[3 * L + a]))
        return fail(BSSN_EINVAL,
                    "level %d: points are not a quarter coarse spacing from "
                    "level %d's along axis %d",
                    L, L - 1, a);
    }
  }
  std::vector<Lat> lat(npatch);
  for (int p = 0; p < npatch; ++p) {
    const bssn_grid& G = patches[p].grid;
    const bssn_grid& R = patches[first[patches[p].level]].grid;
    Lat& l = lat[p];
    l.level = patches[p].level;
    l.g = G.ghost;
    l.st[0] = 1;
    l.st[1] = G.sy;
    l.st[2] = G.sz;
    for (int a = 0; a < 3; ++a) {
      l.n[a] = G.n[a];
      if (std::fabs(G.h[a] - R.h[a]) > 1e-12 * R.h[a])
        return fail(BSSN_EINVAL, "patch %d: h[%d] differs from its level's",
                    p, a);
      if (!near_int((G.origin[a] - R.origin[a]) / R.h[a], &l.off[a]))
        return fail(BSSN_EINVAL,
                    "patch %d: origin not on its level's lattice (axis %d)",
                    p, a);
    }
  }

  std::vector<AmrOp> ops;
  std::vector<AmrTile> tiles;
  bssn_amr_plan plan;
  plan.npatch = npatch;
  plan.nlevel = nlevel;
  plan.fill_begin.assign(nlevel, 0);
  plan.fill_count.assign(nlevel, 0);
  plan.tile_begin.assign(nlevel, 0);
  plan.tile_count.assign(nlevel, 0);
  plan.nprolong.assign(nlevel, 0);
  plan.restr_begin.assign(nlevel, 0);
  plan.restr_count.assign(nlevel, 0);
  for (int L = 0; L < nlevel; ++L) {
    plan.fill_begin[L] = int64_t(ops.size());
    plan.tile_begin[L] = int64_t(tiles.size());
    for (int p = 0; p < npatch; ++p) {
      const Lat& P = lat[p];
      if (P.level != L) continue;
      std::map<std::array<int64_t, 4>, TileAcc> acc;  // (box z, y, x, c)
      int64_t idx[3];
      for (idx[2] = 0; idx[2] < P.n[2] + 2 * P.g; ++idx[2])
        for (idx[1] = 0; idx[1] < P.n[1] + 2 * P.g; ++idx[1])
          for (idx[0] = 0; idx[0] < P.n[0] + 2 * P.g; ++idx[0]) {
            bool inner = true;
            int64_t G[3];
            for (int a = 0; a < 3; ++a) {
              inner = inner && idx[a] >= P.g && idx[a] < P.g + P.n[a];
              G[a] = P.off[a] + idx[a] - P.g;
            }
            if (inner) continue;
            AmrOp op{};
            op.dst = storage(P, idx);
            op.dpatch = p;
            bool found = false;
            for (int q = 0; q < npatch && !found; ++q) {
              const Lat& Q = lat[q];
              if (q == p || Q.level != L) continue;
              int64_t s[3];
              bool in = true;
              for (int a = 0; a < 3; ++a) {
                in = in && G[a] >= Q.off[a] && G[a] < Q.off[a] + Q.n[a];
                s[a] = G[a] - Q.off[a] + Q.g;
              }
              if (!in) continue;
              op.src = storage(Q, s);
              op.spatch = q;
              op.code = 0;
              found = true;
            }
            if (found) {
              ops.push_back(op);
              continue;
            }
            if (L == 0) continue;  // physical boundary
            for (int c = 0; c < npatch && !found; ++c) {
              const Lat& C = lat[c];
              if (C.level != L - 1) continue;
              int64_t b[3];
              bool in = true;
              for (int a = 0; a < 3; ++a) {
                const int64_t q = 2 * D[3 * L + a] + G[a];
                b[a] = floordiv(q - 1, 2) - 1 - C.off[a] + C.g;
                in = in && b[a] >= 0 && b[a] + 3 <= C.n[a] + 2 * C.g - 1;
              }
              if (!in) continue;
              TileAcc& T = acc[{idx[2] / 8, idx[1] / 8, idx[0] / 8, c}];
              const int pt = int(idx[0] % 8 + 8 * (idx[1] % 8) +
                                 64 * (idx[2] % 8));
              T.mask[pt >> 6] |= uint64_t(1) << (pt & 63);
              for (int a = 0; a < 3; ++a) {
                T.bmin[a] = b[a] < T.bmin[a] ? b[a] : T.bmin[a];
                T.bmax[a] = b[a] > T.bmax[a] ? b[a] : T.bmax[a];
                const int e = int(idx[a] % 8);
                T.lo[a] = e < T.lo[a] ? e : T.lo[a];
                T.hi[a] = e > T.hi[a] ? e : T.hi[a];
              }
              ++plan.nprolong[L];
              found = true;
            }
            if (!found)
              return fail(BSSN_EINVAL,
                          "patch %d (level %d): ghost point (%lld, %lld, "
                          "%lld) lies in no sibling interior and no coarse "
                          "patch holds its interpolation block",
                          p, L, (long long)idx[0], (long long)idx[1],
                          (long long)idx[2]);
          }
      for (const auto& kv : acc) {
        const int c = int(kv.first[3]);
        const Lat& C = lat[c];
        const TileAcc& A = kv.second;
        AmrTile t{};
        t.dpatch = p;
        t.spatch = c;
        int64_t o[3] = {kv.first[2] * 8, kv.first[1] * 8, kv.first[0] * 8};
        for (int a = 0; a < 3; ++a) {
          t.c[a] = uint8_t(A.bmax[a] - A.bmin[a] + 4);
          t.lo[a] = uint8_t(A.lo[a]);
          t.m[a] = uint8_t(A.hi[a] - A.lo[a] + 1);
          const int64_t q0 = 2 * D[3 * L + a] + P.off[a] + o[a] - P.g;
          const int64_t f0 = floordiv(q0 - 1, 2);
          const int64_t e0 = q0 - 1 - 2 * f0;
          t.r0[a] = int32_t(f0 - 1 - C.off[a] + C.g - A.bmin[a]);
          t.code |= int32_t(e0) << a;
        }
        for (int w = 0; w < 8; ++w) t.mask[w] = A.mask[w];
        t.dst0 = storage(P, o);
        t.src0 = storage(C, A.bmin);
        tiles.push_back(t);
      }
    }
    plan.fill_count[L] = int64_t(ops.size()) - plan.fill_begin[L];
    plan.tile_count[L] = int64_t(tiles.size()) - plan.tile_begin[L];
  }
  for (int L = 1; L < nlevel; ++L) {
    plan.restr_begin[L] = int64_t(ops.size());
    for (int c = 0; c < npatch; ++c) {
      const Lat& C = lat[c];
      if (C.level != L - 1) continue;
      int64_t idx[3];
      for (idx[2] = C.g; idx[2] < C.g + C.n[2]; ++idx[2])
        for (idx[1] = C.g; idx[1] < C.g + C.n[1]; ++idx[1])
          for (idx[0] = C.g; idx[0] < C.g + C.n[0]; ++idx[0]) {
            int64_t F[3];
            for (int a = 0; a < 3; ++a)
              F[a] = 2 * (C.off[a] + idx[a] - C.g - D[3 * L + a]);
            for (int f = 0; f < npatch; ++f) {
              const Lat& Fp = lat[f];
              if (Fp.level != L) continue;
              bool in = true;
              int64_t b[3];
              for (int a = 0; a < 3; ++a) {
                in = in && F[a] >= Fp.off[a] &&
                     F[a] + 1 < Fp.off[a] + Fp.n[a];
                b[a] = F[a] - Fp.off[a] + Fp.g - 1;
              }
              if (!in) continue;
              AmrOp op{};
              op.dst = storage(C, idx);
              op.dpatch = c;
              op.src = storage(Fp, b);
              op.spatch = f;
              op.code = 0;
              ops.push_back(op);
              break;
            }
          }
    }
    plan.restr_count[L] = int64_t(ops.size()) - plan.restr_begin[L];
  }

  std::vector<AmrGeo> geo(npatch);
  for (int p = 0; p < npatch; ++p)
    geo[p] = AmrGeo{patches[p].grid.sy, patches[p].grid.sz,
                    patches[p].grid.sf};
  hipError_t e = hipGetDevice(&plan.device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  auto* P = new bssn_amr_plan(std::move(plan));
  e = hipMalloc((void**)&P->d_geo, sizeof(AmrGeo) * npatch);
  if (e == hipSuccess && !ops.empty())
    e = hipMalloc((void**)&P->d_ops, sizeof(AmrOp) * ops.size());
  if (e == hipSuccess)
    e = hipMemcpy(P->d_geo, geo.data(), sizeof(AmrGeo) * npatch,
                  hipMemcpyHostToDevice);
  if (e == hipSuccess && !ops.empty())
    e = hipMemcpy(P->d_ops, ops.data(), sizeof(AmrOp) * ops.size(),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess && !tiles.empty())
    e = hipMalloc((void**)&P->d_tiles, sizeof(AmrTile) * tiles.size());
  if (e == hipSuccess && !tiles.empty())
    e = hipMemcpy(P->d_tiles, tiles.data(), sizeof(AmrTile) * tiles.size(),
                  hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    bssn_amr_plan_destroy(P);
    return hip_fail(e, "bssn_amr_plan_create upload");
  }
  *out = P;
  return BSSN_OK;
}

int bssn_amr_plan_counts(const bssn_amr_plan* plan, int level,
                         int64_t* counts) {
  if (!plan || !counts) return fail(BSSN_EINVAL, "plan or counts is NULL");
  if (level < 0 || level >= plan->nlevel)
    return fail(BSSN_EINVAL, "level %d outside 0..%d", level,
                plan->nlevel - 1);
  counts[0] = plan->fill_count[level] + plan->nprolong[level];
  counts[1] = plan->fill_count[level];
  counts[2] = plan->restr_count[level];
  return BSSN_OK;
}

static int check_level_call(const bssn_amr_plan* plan, int level, int lo) {
  if (!plan) return fail(BSSN_EINVAL, "plan is NULL");
  if (level < lo || level >= plan->nlevel)
    return fail(BSSN_EINVAL, "level %d outside %d..%d", level, lo,
                plan->nlevel - 1);
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != plan->device)
    return fail(BSSN_EINVAL, "plan built on device %d, current device %d",
                plan->device, dev);
  return BSSN_OK;
}

int bssn_amr_fill_ghosts(const bssn_amr_plan* plan, int level,
                         double* const* u_tab, int ntl,
                         const double* const* const* src_tabs,
                         const double* t_src, double t, void* stream) {
  if (!plan) return fail(BSSN_EINVAL, "plan is NULL");
  if (!u_tab) return fail(BSSN_EINVAL, "u_tab is NULL");
  AmrTime T{};
  if (level == 0) {  // sibling exchange only: no coarse level
    int rc = check_level_call(plan, 0, 0);
    if (rc) return rc;
    hipError_t e = launch_amr_fill(plan->d_ops + plan->fill_begin[0],
                                   plan->fill_count[0], plan->d_geo, u_tab,
                                   (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "bssn_amr_fill_ghosts launch");
    return BSSN_OK;
  }
  if (!src_tabs || !t_src)
    return fail(BSSN_EINVAL, "src_tabs and t_src must be non-NULL");
  if (ntl < 1 || ntl > 3)
    return fail(BSSN_EINVAL, "ntl = %d outside 1..3", ntl);
  if (!std::isfinite(t)) return fail(BSSN_EINVAL, "t is not finite");
  T.ntl = ntl;
  for (int l = 0; l < ntl; ++l) {
    if (!src_tabs[l]) return fail(BSSN_EINVAL, "src_tabs[%d] is NULL", l);
    if (!std::isfinite(t_src[l]))
      return fail(BSSN_EINVAL, "t_src[%d] is not finite", l);
    for (int m = 0; m < l; ++m)
      if (t_src[m] == t_src[l])
        return fail(BSSN_EINVAL, "t_src[%d] == t_src[%d]", m, l);
  }
  int rc = check_level_call(plan, level, 1);
  if (rc) return rc;
  // Lagrange weights in time through the coarse time levels
  for (int l = 0; l < ntl; ++l) {
    double w = 1.0;
    for (int m = 0; m < ntl; ++m)
      if (m != l) w *= (t - t_src[m]) / (t_src[l] - t_src[m]);
    T.tab[l] = src_tabs[l];
    T.w[l] = w;
  }
  hipError_t e = launch_amr_fill(plan->d_ops + plan->fill_begin[level],
                                 plan->fill_count[level], plan->d_geo, u_tab,
                                 (hipStream_t)stream);
  if (e == hipSuccess)
    e = launch_amr_prolong(plan->d_tiles + plan->tile_begin[level],
                           plan->tile_count[level], plan->d_geo, u_tab, T,
                           (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "bssn_amr_fill_ghosts launch");
  return BSSN_OK;
}

int bssn_amr_restrict(const bssn_amr_plan* plan, int level,
                      const double* const* fine_tab, double* const* coarse_tab,
                      void* stream) {
  if (!plan) return fail(BSSN_EINVAL, "plan is NULL");
  if (!fine_tab || !coarse_tab)
    return fail(BSSN_EINVAL, "fine_tab and coarse_tab must be non-NULL");
  int rc = check_level_call(plan, level, 1);
  if (rc) return rc;
  hipError_t e = launch_amr_restrict(
      plan->d_ops + plan->restr_begin[level], plan->restr_count[level],
      plan->d_geo, coarse_tab, fine_tab, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "bssn_amr_restrict launch");
  return BSSN_OK;
}

int bssn_amr_plan_destroy(bssn_amr_plan* plan) {
  if (!plan) return BSSN_OK;
  if (plan->d_ops) (void)hipFree(plan->d_ops);
  if (plan->d_tiles) (void)hipFree(plan->d_tiles);
  if (plan->d_geo) (void)hipFree(plan->d_geo);
  delete plan;
  return BSSN_OK;
}

}  // extern "C"
