// bssn_kernels.h -- host-side launchers implemented in the .hip files.
#pragma once
#include <hip/hip_runtime.h>

#include "bssn_internal.h"

namespace bssn {

// One RK4 stage (or the bare RHS for stage ST_RHS) on one patch.
// precision 0: FP64; 1: FP32 tiles + FP64 tiles (two launches).  With
// kout set, the right-hand side at the outermost layer of interior points
// (the radiative boundary's roots) also goes to kout (state layout):
// stored by the LDS kernels from their own tiles, or by the shell kernel
// (FP64) before a direct-kernel stage.
// Kernel choice: PATH_AUTO uses the LDS-pipelined persistent kernel for
// static grids whose layout allows 16-byte granules, the direct-load kernel
// otherwise; PATH_DIRECT forces the direct-load kernel.
enum : int { PATH_AUTO = 0, PATH_DIRECT = 1 };
hipError_t launch_stage_o4(const Patch& P, const Gauge& G, int periodic,
                           int stage, int precision, int path, int nwg,
                           hipStream_t st, double* kout = nullptr);
hipError_t launch_stage_o8(const Patch& P, const Gauge& G, int periodic,
                           int stage, int precision, int path, int nwg,
                           hipStream_t st, double* kout = nullptr);
int stage_path();          // current PATH_* (bssn_set_path)
int persistent_groups();   // workgroups of a persistent launch (CU count)
inline hipError_t launch_stage(const Patch& P, const Gauge& G, int order,
                               int periodic, int stage, int precision,
                               hipStream_t st, double* kout = nullptr) {
  const int path = stage_path(), nwg = persistent_groups();
  return order == 8 ? launch_stage_o8(P, G, periodic, stage, precision, path,
                                      nwg, st, kout)
                    : launch_stage_o4(P, G, periodic, stage, precision, path,
                                      nwg, st, kout);
}

// One static patch with an explicit kernel variant (VAR_*); nwg bounds the
// persistent launch of VAR_LDS.
hipError_t launch_patch_o4(const Patch& P, const Gauge& G, int stage,
                           int precision, int variant, int nwg,
                           hipStream_t st);
hipError_t launch_patch_o8(const Patch& P, const Gauge& G, int stage,
                           int precision, int variant, int nwg,
                           hipStream_t st);
// Whether the layout of P (every buffer it names) allows the variant.
bool variant_ok_o4(const Patch& P, int variant);
bool variant_ok_o8(const Patch& P, int variant);

// One batched launch over device work lists.  VAR_LDS: items are LdsItem,
// workgroup q runs items [wstart[q], wstart[q+1]), nwg workgroups (in mixed
// precision: the FP32 launch, then the FP64 pass over cand).  VAR_D*:
// items are DirectItem, one workgroup per item.
struct BatchLaunch {
  int variant;
  const Patch* patches;   // device, indexed by item.patch
  const void* items;      // device
  const int32_t* wstart;  // device, nwg + 1 entries (VAR_LDS)
  int nitems;
  int nwg;
  // VAR_LDS, mixed precision: every tile of the launch's patches once, in
  // a scattering order; the FP64 pass examines them (device, ncand)
  const TileRef* cand;
  int ncand;
};
hipError_t launch_batch_o4(const BatchLaunch& B, const Gauge& G, int stage,
                           int precision, hipStream_t st);
hipError_t launch_batch_o8(const BatchLaunch& B, const Gauge& G, int stage,
                           int precision, hipStream_t st);
inline hipError_t launch_patch(const Patch& P, const Gauge& G, int order,
                               int stage, int precision, int variant,
                               int nwg, hipStream_t st) {
  return order == 8
             ? launch_patch_o8(P, G, stage, precision, variant, nwg, st)
             : launch_patch_o4(P, G, stage, precision, variant, nwg, st);
}
inline bool variant_ok(const Patch& P, int order, int variant) {
  return order == 8 ? variant_ok_o8(P, variant) : variant_ok_o4(P, variant);
}
inline hipError_t launch_batch(const BatchLaunch& B, const Gauge& G,
                               int order, int stage, int precision,
                               hipStream_t st) {
  return order == 8 ? launch_batch_o8(B, G, stage, precision, st)
                    : launch_batch_o4(B, G, stage, precision, st);
}

// Constraint fields and norms (see bssn_constraints in bssn.h).
struct ConstraintArgs {
  const double* u;
  double* H;
  double* M;
  double* Gc;
  int32_t n[3];
  int32_t ghost;
  int32_t sy, sz;
  int64_t sf;
  double origin[3];
  double h[3];
  int32_t periodic;
  int32_t ncent;
  double centres[16][3];
  double r_exc;
};
hipError_t launch_constraints(const ConstraintArgs& A, int order,
                              double* partials, int nblocks_max,
                              double* norms, hipStream_t st);
int constraint_blocks(const ConstraintArgs& A);

// Radiative outer boundary (bssn_radiative_rhs): the right-hand side on the
// ghost layers of rhs from the state u and the interior of rhs.
struct RadiativeArgs {
  const double* u;
  double* rhs;
  int32_t n[3];
  int32_t ghost;
  int64_t sy, sz, sf;
  double origin[3];
  double h[3];
  double i2h[3];  // 1 / (2 h), per axis
  double x0[NSLOT];
  double v0[NSLOT];
  int32_t power;
};
hipError_t launch_radiative(const RadiativeArgs& A, hipStream_t st);
// The radiative boundary inside an RK4 stage: the same right-hand side at
// every ghost point (from A.u = the stage input and A.rhs = a buffer whose
// outermost interior layer holds the interior right-hand side), fed
// straight into the stage update of that point (as the fused stage does for
// interior points): acc and out at the ghost points.
struct RadStage {
  const double* u_n;
  double* acc;
  double* out;
  double dt;
  int32_t stage;
};
hipError_t launch_radiative_stage(const RadiativeArgs& A, const RadStage& S,
                                  hipStream_t st);

// ADM -> BSSN initial conversion (bssn_from_adm): adm holds 16 slots in
// the state layout (g_ij, K_ij, alpha, beta^i); every slot of u is written
// at every storage point.
struct AdmArgs {
  const double* adm;
  double* u;
  int32_t n[3];
  int32_t ghost;
  int64_t sy, sz, sf;
  double h[3];
  int32_t order;
};
hipError_t launch_from_adm(const AdmArgs& A, hipStream_t st);

// Puncture tracking (bssn_track_punctures): the state's shift at each
// position (tricubic), one Euler step of dx/dt = -beta.
struct TrackArgs {
  const double* u;
  int32_t n[3];
  int32_t ghost;
  int64_t sy, sz, sf;
  double origin[3];
  double h[3];
};
hipError_t launch_track(const TrackArgs& A, double* pos, int np, double dt,
                        hipStream_t st);

// Multipole coefficients on a coordinate sphere (bssn_multipole).
struct MultipoleArgs {
  const double* re;  // field slots, element 0 of the storage grid
  const double* im;  // may be null
  int32_t n[3];
  int32_t ghost;
  int64_t sy, sz;
  double origin[3], h[3];
  double centre[3];
  double radius;
  int32_t spin, lmax, ntheta, nphi;
};
// Point chunks per (l, m) (at most 64): the partial sums take
// 2 (lmax + 1)^2 chunks doubles of the workspace after the point values.
inline int multipole_chunks(int ntheta, int nphi) {
  const int c = (ntheta * nphi + 255) / 256;
  return c < 64 ? c : 64;
}
hipError_t launch_multipole(const MultipoleArgs& A, double* work,
                            double* coeffs, hipStream_t st);

// The Weyl scalar Psi_4 (bssn_psi4): re and im at the interior points of
// out (slots 0 and 1 of the grid's layout) from the state u.
struct Psi4Args {
  const double* u;
  double* out;
  int32_t n[3];
  int32_t ghost;
  int64_t sy, sz, sf;
  double origin[3], h[3];
  double centre[3];
};
hipError_t launch_psi4(const Psi4Args& A, int order, hipStream_t st);

// Mesh-refinement glue (bssn_amr_*): ops built on the host, one per copied
// ghost point or restricted coarse point.  dst and src are element offsets
// from the slot-0 origin of the destination and source patch states.
struct AmrOp {
  int64_t dst, src;
  int32_t dpatch, spatch;
  int32_t code, pad;
};
struct AmrGeo {
  int64_t sy, sz, sf;
};
struct AmrTime {
  const double* const* tab[3];  // device tables of coarse state pointers
  double w[3];                  // Lagrange weights in time
  int ntl;
};
// Prolonged ghost points grouped by 8 x 8 x 8 box of the fine storage grid
// and coarse source patch: the coarse region the box's points read (at
// most 8 per axis) is staged in LDS once per (tile, slot, time level).
struct AmrTile {
  int64_t dst0, src0;  // box origin in dpatch; region origin in spatch
  int32_t dpatch, spatch;
  int32_t r0[3];       // block base of box point 0, relative to the region
  int32_t code;        // bit a: (q - 1) mod 2 of box point 0 along axis a
  uint8_t c[3];        // region extents (4..8)
  uint8_t lo[3], m[3]; // bounding box of the filled points: first, extent
  uint8_t pad[7];
  uint64_t mask[8];    // point i + 8 j + 64 k of the box is filled
};
hipError_t launch_amr_fill(const AmrOp* ops, int64_t nops, const AmrGeo* geo,
                           double* const* u, hipStream_t st);
hipError_t launch_amr_prolong(const AmrTile* tiles, int64_t ntiles,
                              const AmrGeo* geo, double* const* u,
                              const AmrTime& T, hipStream_t st);
hipError_t launch_amr_restrict(const AmrOp* ops, int64_t nops,
                               const AmrGeo* geo, double* const* coarse,
                               const double* const* fine, hipStream_t st);

// Count of tiles whose minimum lapse is below thr (device counter), over
// the tiles of the LDS kernel (lds = 1) or of the direct kernel.
hipError_t launch_tile_count(const Patch& P, double thr, int lds,
                             unsigned long long* counter, hipStream_t st);
void tile_grid(const Patch& P, int lds, dim3& grd, dim3& blk);

}  // namespace bssn
