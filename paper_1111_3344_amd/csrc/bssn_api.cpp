// bssn_api.cpp -- the extern "C" entry points of include/bssn.h: argument
// validation (before anything is enqueued), error reporting and dispatch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bssn.h"
#include "bssn_api_internal.h"
#include "bssn_internal.h"
#include "bssn_kernels.h"

namespace bssn {

static thread_local std::string g_err = "no error";

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(BSSN_EHIP, "%s: %s", what, hipGetErrorString(e));
}

int check_grid(const bssn_grid* g, int order) {
  if (!g) return fail(BSSN_EINVAL, "grid is NULL");
  const int need = order == 8 ? 5 : 3;
  for (int a = 0; a < 3; ++a) {
    if (g->n[a] < 1) return fail(BSSN_EINVAL, "grid.n[%d] = %d < 1", a, g->n[a]);
    if (!(g->h[a] > 0.0) || !std::isfinite(g->h[a]))
      return fail(BSSN_EINVAL, "grid.h[%d] must be finite and > 0", a);
    if (!std::isfinite(g->origin[a]))
      return fail(BSSN_EINVAL, "grid.origin[%d] is not finite", a);
  }
  if (g->ghost < need)
    return fail(BSSN_EINVAL, "grid.ghost = %d < %d required by order %d",
                g->ghost, need, order);
  if (g->bc != BSSN_BC_STATIC && g->bc != BSSN_BC_PERIODIC)
    return fail(BSSN_EINVAL, "grid.bc = %d is not a BSSN_BC_* value", g->bc);
  if (g->bc == BSSN_BC_PERIODIC)
    for (int a = 0; a < 3; ++a)
      if (g->n[a] < need)
        return fail(BSSN_EINVAL,
                    "periodic grid.n[%d] = %d below the stencil reach %d", a,
                    g->n[a], need);
  const int64_t ex = g->n[0] + 2LL * g->ghost, ey = g->n[1] + 2LL * g->ghost,
                ez = g->n[2] + 2LL * g->ghost;
  if (g->sy < ex) return fail(BSSN_EINVAL, "grid.sy < n[0] + 2 ghost");
  if (g->sz < g->sy * ey) return fail(BSSN_EINVAL, "grid.sz < sy (n[1] + 2 ghost)");
  if (g->sf < g->sz * ez) return fail(BSSN_EINVAL, "grid.sf < sz (n[2] + 2 ghost)");
  if (g->sf * 8 > 0x7fffffffLL)
    return fail(BSSN_EUNSUPPORTED, "one slot exceeds 2 GiB (sf = %lld)",
                (long long)g->sf);
  return BSSN_OK;
}

int check_params(const bssn_params* p) {
  if (!p) return fail(BSSN_EINVAL, "params is NULL");
  if (p->fd_order != 4 && p->fd_order != 8)
    return fail(BSSN_EINVAL, "params.fd_order = %d (4 or 8)", p->fd_order);
  if (p->precision != BSSN_FP64 && p->precision != BSSN_MIXED)
    return fail(BSSN_EINVAL, "params.precision = %d", p->precision);
  const double v[] = {p->ko_eps, p->lapse_f, p->shift_G, p->eta};
  for (double x : v)
    if (!std::isfinite(x)) return fail(BSSN_EINVAL, "non-finite gauge parameter");
  if (p->ko_eps < 0) return fail(BSSN_EINVAL, "params.ko_eps < 0");
  if (std::isnan(p->eta_R)) return fail(BSSN_EINVAL, "params.eta_R is NaN");
  if ((p->lapse_static != 0 && p->lapse_static != 1) ||
      (p->shift_static != 0 && p->shift_static != 1))
    return fail(BSSN_EINVAL, "lapse_static / shift_static must be 0 or 1");
  if (p->precision == BSSN_MIXED && std::isnan(p->fp64_alpha_threshold))
    return fail(BSSN_EINVAL, "fp64_alpha_threshold is NaN");
  return BSSN_OK;
}

Patch make_patch(const bssn_grid* g) {
  Patch P{};
  for (int a = 0; a < 3; ++a) {
    P.n[a] = g->n[a];
    P.origin[a] = g->origin[a];
    P.h[a] = g->h[a];
  }
  for (int a = 0; a < 3; ++a) {
    P.ih[a] = 1.0 / g->h[a];
    P.ih2[a] = 1.0 / (g->h[a] * g->h[a]);
  }
  P.ihm[0] = 1.0 / (g->h[0] * g->h[1]);
  P.ihm[1] = 1.0 / (g->h[0] * g->h[2]);
  P.ihm[2] = 1.0 / (g->h[1] * g->h[2]);
  P.ghost = g->ghost;
  P.sy = int32_t(g->sy);
  P.sz = int32_t(g->sz);
  P.sf = g->sf;
  return P;
}

static int g_path = PATH_AUTO;
int stage_path() { return g_path; }

int persistent_groups() {
  static thread_local int cached_dev = -1, cached_n = 256;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (dev != cached_dev) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount,
                              dev) != hipSuccess || n <= 0)
      n = 256;
    cached_dev = dev;
    cached_n = n;
  }
  return cached_n;
}

Gauge make_gauge(const bssn_params* p) {
  Gauge G{};
  G.ko_eps = p->ko_eps;
  G.lapse_f = p->lapse_f;
  G.shift_G = p->shift_G;
  G.eta = p->eta;
  G.eta_R = (p->eta_R > 0 && std::isfinite(p->eta_R)) ? p->eta_R : 0.0;
  G.lapse_static = p->lapse_static;
  G.shift_static = p->shift_static;
  G.alpha_thr = p->fp64_alpha_threshold;
  return G;
}

}  // namespace bssn

using namespace bssn;

extern "C" {

int bssn_abi_version(void) { return BSSN_ABI_VERSION; }

int bssn_set_path(int path) {
  if (path != BSSN_PATH_AUTO && path != BSSN_PATH_DIRECT)
    return fail(BSSN_EINVAL, "path = %d is not a BSSN_PATH_* value", path);
  g_path = path;
  return BSSN_OK;
}

const char* bssn_last_error(void) { return g_err.c_str(); }

int bssn_rhs(const bssn_grid* grid, const bssn_params* params, const double* u,
             double* rhs, void* stream) {
  int rc = check_params(params);
  if (rc) return rc;
  if ((rc = check_grid(grid, params->fd_order))) return rc;
  if (!u || !rhs) return fail(BSSN_EINVAL, "u and rhs must be non-NULL");
  if (u == rhs) return fail(BSSN_EINVAL, "rhs must not alias u");
  Patch P = make_patch(grid);
  P.u_s = u;
  P.u_n = u;
  P.acc = nullptr;
  P.out = rhs;
  P.dt = 0.0;
  hipError_t e = launch_stage(P, make_gauge(params), params->fd_order,
                              grid->bc == BSSN_BC_PERIODIC, ST_RHS,
                              params->precision, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "bssn_rhs launch");
  g_err = "no error";
  return BSSN_OK;
}

int rk4_stage(const bssn_grid* grid, const bssn_params* params, int stage,
              double dt, const double* u_n, const double* u_s, double* acc,
              double* u_out, void* stream) {
  int rc = check_params(params);
  if (rc) return rc;
  if ((rc = check_grid(grid, params->fd_order))) return rc;
  if (stage < 0 || stage > 3)
    return fail(BSSN_EINVAL, "stage = %d outside 0..3", stage);
  if (!std::isfinite(dt)) return fail(BSSN_EINVAL, "dt is not finite");
  if (!u_n || !u_s || !acc || !u_out)
    return fail(BSSN_EINVAL, "u_n, u_s, acc and u_out must be non-NULL");
  if (u_out == u_s) return fail(BSSN_EINVAL, "u_out must not alias u_s");
  if (acc == u_n || acc == u_s || acc == u_out)
    return fail(BSSN_EINVAL, "acc must not alias any other buffer");
  if (u_out == u_n && stage != 3)
    return fail(BSSN_EINVAL, "u_out may alias u_n only at stage 3");
  Patch P = make_patch(grid);
  P.u_s = u_s;
  P.u_n = u_n;
  P.acc = acc;
  P.out = u_out;
  P.dt = dt;
  hipError_t e = launch_stage(P, make_gauge(params), params->fd_order,
                              grid->bc == BSSN_BC_PERIODIC, stage,
                              params->precision, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "rk4_stage launch");
  g_err = "no error";
  return BSSN_OK;
}

int bssn_from_adm(const bssn_grid* grid, const bssn_params* params,
                  const double* adm, double* u, void* stream) {
  int rc = check_params(params);
  if (rc) return rc;
  if ((rc = check_grid(grid, params->fd_order))) return rc;
  for (int a = 0; a < 3; ++a)
    if (grid->n[a] < 4)
      return fail(BSSN_EINVAL, "grid.n[%d] = %d < 4: the cubic extrapolation "
                  "of the ghost layers reaches 4 points inward", a,
                  grid->n[a]);
  if (!adm || !u) return fail(BSSN_EINVAL, "adm and u must be non-NULL");
  if (adm == u) return fail(BSSN_EINVAL, "u must not alias adm");
  AdmArgs A{};
  A.adm = adm;
  A.u = u;
  for (int a = 0; a < 3; ++a) {
    A.n[a] = grid->n[a];
    A.h[a] = grid->h[a];
  }
  A.ghost = grid->ghost;
  A.sy = grid->sy;
  A.sz = grid->sz;
  A.sf = grid->sf;
  A.order = params->fd_order;
  hipError_t e = launch_from_adm(A, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "bssn_from_adm launch");
  g_err = "no error";
  return BSSN_OK;
}

int bssn_track_punctures(const bssn_grid* grid, const double* u, int npunct,
                         double* pos, double dt, void* stream) {
  int rc = check_grid(grid, 4);
  if (rc) return rc;
  if (!u || !pos) return fail(BSSN_EINVAL, "u and pos must be non-NULL");
  if (npunct < 1 || npunct > 65536)
    return fail(BSSN_EINVAL, "npunct = %d outside 1..65536", npunct);
  if (!std::isfinite(dt)) return fail(BSSN_EINVAL, "dt is not finite");
  TrackArgs A{};
  A.u = u;
  for (int a = 0; a < 3; ++a) {
    A.n[a] = grid->n[a];
    A.origin[a] = grid->origin[a];
    A.h[a] = grid->h[a];
  }
  A.ghost = grid->ghost;
  A.sy = grid->sy;
  A.sz = grid->sz;
  A.sf = grid->sf;
  hipError_t e = launch_track(A, pos, npunct, dt, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "bssn_track_punctures launch");
  g_err = "no error";
  return BSSN_OK;
}

int bssn_multipole(const bssn_grid* grid, const double* re, const double* im,
                   const double* centre, double radius, int spin, int lmax,
                   int ntheta, int nphi, double* work, double* coeffs,
                   void* stream) {
  int rc = check_grid(grid, 4);
  if (rc) return rc;
  if (!re || !work || !coeffs || !centre)
    return fail(BSSN_EINVAL, "re, centre, work and coeffs must be non-NULL");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(centre[a]))
      return fail(BSSN_EINVAL, "centre[%d] is not finite", a);
  if (!(radius > 0.0) || !std::isfinite(radius))
    return fail(BSSN_EINVAL, "radius must be finite and > 0");
  if (spin < -8 || spin > 8) return fail(BSSN_EINVAL, "spin %d outside -8..8", spin);
  if (lmax < 0 || lmax > 16) return fail(BSSN_EINVAL, "lmax %d outside 0..16", lmax);
  if (ntheta < 1 || ntheta > 1024)
    return fail(BSSN_EINVAL, "ntheta %d outside 1..1024", ntheta);
  if (nphi < 1 || nphi > 4096)
    return fail(BSSN_EINVAL, "nphi %d outside 1..4096", nphi);
  MultipoleArgs A{};
  A.re = re;
  A.im = im;
  for (int a = 0; a < 3; ++a) {
    A.n[a] = grid->n[a];
    A.origin[a] = grid->origin[a];
    A.h[a] = grid->h[a];
    A.centre[a] = centre[a];
  }
  A.ghost = grid->ghost;
  A.sy = grid->sy;
  A.sz = grid->sz;
  A.radius = radius;
  A.spin = spin;
  A.lmax = lmax;
  A.ntheta = ntheta;
  A.nphi = nphi;
  hipError_t e = launch_multipole(A, work, coeffs, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "bssn_multipole launch");
  g_err = "no error";
  return BSSN_OK;
}

int bssn_psi4(const bssn_grid* grid, int fd_order, const double* u,
              const double* centre, double* psi4, void* stream) {
  if (fd_order != 4 && fd_order != 8)
    return fail(BSSN_EINVAL, "fd_order = %d (4 or 8)", fd_order);
  int rc = check_grid(grid, fd_order);
  if (rc) return rc;
  if (!u || !psi4 || !centre)
    return fail(BSSN_EINVAL, "u, centre and psi4 must be non-NULL");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(centre[a]))
      return fail(BSSN_EINVAL, "centre[%d] is not finite", a);
  // the two output slots [psi4, psi4 + 2 sf) must not overlap the state
  // [u, u + 25 sf)
  const uintptr_t o0 = (uintptr_t)psi4, o1 = o0 + 16 * (uintptr_t)grid->sf;
  const uintptr_t u0 = (uintptr_t)u, u1 = u0 + 8 * (uintptr_t)grid->sf * 25;
  if (o0 < u1 && u0 < o1)
    return fail(BSSN_EINVAL, "psi4 overlaps the state u");
  Psi4Args A{};
  A.u = u;
  A.out = psi4;
  for (int a = 0; a < 3; ++a) {
    A.n[a] = grid->n[a];
    A.origin[a] = grid->origin[a];
    A.h[a] = grid->h[a];
    A.centre[a] = centre[a];
  }
  A.ghost = grid->ghost;
  A.sy = grid->sy;
  A.sz = grid->sz;
  A.sf = grid->sf;
  hipError_t e = launch_psi4(A, fd_order, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "bssn_psi4 launch");
  g_err = "no error";
  return BSSN_OK;
}

namespace {
// Checks shared by the radiative entry points, and their kernel arguments.
int radiative_args(const bssn_grid* grid, const double* x0, const double* v0,
                   int power, const double* u, double* rhs, RadiativeArgs& A) {
  if (grid->bc != BSSN_BC_STATIC)
    return fail(BSSN_EINVAL, "the radiative boundary needs a static grid "
                "(its ghost layers are the boundary points)");
  if (!x0 || !v0) return fail(BSSN_EINVAL, "x0 and v0 must be non-NULL");
  if (power < 0 || power > 16)
    return fail(BSSN_EINVAL, "power = %d outside 0..16", power);
  for (int s = 0; s < BSSN_NSLOT; ++s)
    if (!std::isfinite(x0[s]) || !std::isfinite(v0[s]) || v0[s] < 0.0)
      return fail(BSSN_EINVAL, "slot %d: x0 and v0 must be finite, v0 >= 0",
                  s);
  // r = 0 at a boundary point or at one of the interior points the
  // boundary is carried from (the outermost interior layer) would divide by
  // zero: the coordinate origin must be neither
  bool at[3];
  bool deep = true;
  for (int a = 0; a < 3; ++a) {
    const double j = grid->ghost - grid->origin[a] / grid->h[a];
    const double jr = std::nearbyint(j);
    at[a] = std::fabs(j - jr) <= 1e-9 * (1.0 + std::fabs(j)) && jr >= 0 &&
            jr < grid->n[a] + 2.0 * grid->ghost;
    deep = deep && jr > grid->ghost && jr < grid->n[a] + grid->ghost - 1;
  }
  if (at[0] && at[1] && at[2] && !deep)
    return fail(BSSN_EINVAL, "the coordinate origin is a boundary point or "
                "on the outermost interior layer");
  A = RadiativeArgs{};
  A.u = u;
  A.rhs = rhs;
  for (int a = 0; a < 3; ++a) {
    A.n[a] = grid->n[a];
    A.origin[a] = grid->origin[a];
    A.h[a] = grid->h[a];
    A.i2h[a] = 1.0 / (2.0 * grid->h[a]);
  }
  A.ghost = grid->ghost;
  A.sy = grid->sy;
  A.sz = grid->sz;
  A.sf = grid->sf;
  for (int s = 0; s < BSSN_NSLOT; ++s) {
    A.x0[s] = x0[s];
    A.v0[s] = v0[s];
  }
  A.power = power;
  return BSSN_OK;
}
}  // namespace

int bssn_radiative_rhs(const bssn_grid* grid, const double* x0,
                       const double* v0, int power, const double* u,
                       double* rhs, void* stream) {
  int rc = check_grid(grid, 4);
  if (rc) return rc;
  if (!u || !rhs) return fail(BSSN_EINVAL, "u and rhs must be non-NULL");
  if (u == rhs) return fail(BSSN_EINVAL, "rhs must not alias u");
  RadiativeArgs A;
  if ((rc = radiative_args(grid, x0, v0, power, u, rhs, A))) return rc;
  hipError_t e = launch_radiative(A, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "bssn_radiative_rhs launch");
  g_err = "no error";
  return BSSN_OK;
}

int rk4_stage_radiative(const bssn_grid* grid, const bssn_params* params,
                        int stage, double dt, const double* x0,
                        const double* v0, int power, const double* u_n,
                        const double* u_s, double* acc, double* u_out,
                        double* k, void* stream) {
  int rc = check_params(params);
  if (rc) return rc;
  if ((rc = check_grid(grid, params->fd_order))) return rc;
  if (stage < 0 || stage > 3)
    return fail(BSSN_EINVAL, "stage = %d outside 0..3", stage);
  if (!std::isfinite(dt)) return fail(BSSN_EINVAL, "dt is not finite");
  if (!u_n || !u_s || !acc || !u_out || !k)
    return fail(BSSN_EINVAL, "u_n, u_s, acc, u_out and k must be non-NULL");
  if (u_out == u_s) return fail(BSSN_EINVAL, "u_out must not alias u_s");
  if (acc == u_n || acc == u_s || acc == u_out)
    return fail(BSSN_EINVAL, "acc must not alias any other buffer");
  if (u_out == u_n && stage != 3)
    return fail(BSSN_EINVAL, "u_out may alias u_n only at stage 3");
  if (k == u_n || k == u_s || k == acc || k == u_out)
    return fail(BSSN_EINVAL, "k must not alias any other buffer");
  RadiativeArgs A;
  if ((rc = radiative_args(grid, x0, v0, power, u_s, k, A))) return rc;
  const hipStream_t st = (hipStream_t)stream;
  const Gauge G = make_gauge(params);
  // 1. the fused stage at the interior points; it also leaves the
  //    right-hand side of the outermost interior layer (the radiative
  //    boundary's roots) in k
  Patch P = make_patch(grid);
  P.u_s = u_s;
  P.u_n = u_n;
  P.acc = acc;
  P.out = u_out;
  P.dt = dt;
  hipError_t e = launch_stage(P, G, params->fd_order, 0, stage,
                              params->precision, st, k);
  if (e != hipSuccess) return hip_fail(e, "rk4_stage_radiative launch");
  // 2. the boundary points: radiative right-hand side and stage update
  RadStage R{u_n, acc, u_out, dt, stage};
  e = launch_radiative_stage(A, R, st);
  if (e != hipSuccess)
    return hip_fail(e, "rk4_stage_radiative boundary launch");
  g_err = "no error";
  return BSSN_OK;
}

}  // extern "C"

// ---- workspaces that live until the process ends ---------------------------------
namespace bssn {
// Validation of the bssn_constraints arguments and the kernels' view of them.
int constraint_args(const bssn_grid* grid, const bssn_params* params,
                    const double* u, double* H, double* M, double* G,
                    const double* centres, int ncent, double r_exc,
                    const double* norms, ConstraintArgs* A) {
  int rc = check_params(params);
  if (rc) return rc;
  if ((rc = check_grid(grid, params->fd_order))) return rc;
  if (!u || !norms) return fail(BSSN_EINVAL, "u and norms must be non-NULL");
  if (ncent < 0 || ncent > 16)
    return fail(BSSN_EINVAL, "ncent = %d outside 0..16", ncent);
  if (ncent > 0 && !centres)
    return fail(BSSN_EINVAL, "centres is NULL with ncent > 0");
  if (std::isnan(r_exc)) return fail(BSSN_EINVAL, "r_exc is NaN");
  const double* outs[3] = {H, M, G};
  for (const double* o : outs)
    if (o && o == u) return fail(BSSN_EINVAL, "outputs must not alias u");
  *A = ConstraintArgs{};
  A->u = u;
  A->H = H;
  A->M = M;
  A->Gc = G;
  for (int a = 0; a < 3; ++a) {
    A->n[a] = grid->n[a];
    A->origin[a] = grid->origin[a];
    A->h[a] = grid->h[a];
  }
  A->ghost = grid->ghost;
  A->sy = int32_t(grid->sy);
  A->sz = int32_t(grid->sz);
  A->sf = grid->sf;
  A->periodic = grid->bc == BSSN_BC_PERIODIC;
  A->ncent = ncent;
  for (int c = 0; c < ncent; ++c)
    for (int a = 0; a < 3; ++a) A->centres[c][a] = centres[3 * c + a];
  A->r_exc = r_exc;
  return BSSN_OK;
}

namespace {
struct DeviceWs {
  double* partials = nullptr;
  size_t partials_n = 0;  // records of 8 doubles
  unsigned long long* counter = nullptr;
};
std::mutex g_ws_mu;
std::vector<DeviceWs> g_ws;

int device_ws(DeviceWs** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_ws_mu);
  if ((int)g_ws.size() <= dev) g_ws.resize(dev + 1);
  *out = &g_ws[dev];
  return BSSN_OK;
}
}  // namespace
}  // namespace bssn

extern "C" {

int bssn_constraints(const bssn_grid* grid, const bssn_params* params,
                     const double* u, double* H, double* M, double* G,
                     const double* centres, int ncent, double r_exc,
                     double* norms, void* stream) {
  ConstraintArgs A{};
  int rc = constraint_args(grid, params, u, H, M, G, centres, ncent, r_exc,
                           norms, &A);
  if (rc) return rc;
  DeviceWs* ws = nullptr;
  if ((rc = device_ws(&ws))) return rc;
  const size_t nb = size_t(constraint_blocks(A));
  {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    if (ws->partials_n < nb) {
      // the old workspace may still be read by enqueued work
      hipError_t e = hipDeviceSynchronize();
      if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
      if (ws->partials) (void)hipFree(ws->partials);
      ws->partials = nullptr;
      ws->partials_n = 0;
      const size_t want = nb < 65536 ? 65536 : nb;
      e = hipMalloc((void**)&ws->partials, want * 8 * sizeof(double));
      if (e != hipSuccess) return fail(BSSN_ENOMEM, "workspace: %s", hipGetErrorString(e));
      ws->partials_n = want;
    }
  }
  hipError_t e = launch_constraints(A, params->fd_order, ws->partials,
                                    int(ws->partials_n), norms,
                                    (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "bssn_constraints launch");
  g_err = "no error";
  return BSSN_OK;
}

int bssn_mixed_tile_count(const bssn_grid* grid, const bssn_params* params,
                          const double* u, int64_t* n_fp64, int64_t* n_tiles,
                          void* stream) {
  int rc = check_params(params);
  if (rc) return rc;
  if ((rc = check_grid(grid, params->fd_order))) return rc;
  if (!u || !n_fp64 || !n_tiles)
    return fail(BSSN_EINVAL, "u, n_fp64 and n_tiles must be non-NULL");
  DeviceWs* ws = nullptr;
  if ((rc = device_ws(&ws))) return rc;
  hipStream_t st = (hipStream_t)stream;
  {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    if (!ws->counter) {
      hipError_t e = hipMalloc((void**)&ws->counter, sizeof(unsigned long long));
      if (e != hipSuccess) return fail(BSSN_ENOMEM, "counter: %s", hipGetErrorString(e));
    }
  }
  Patch P = make_patch(grid);
  P.u_s = u;
  // the tiles of the kernel a stage on this grid runs
  const int lds = grid->bc == BSSN_BC_STATIC && stage_path() == PATH_AUTO &&
                  variant_ok(P, params->fd_order, VAR_LDS);
  hipError_t e = hipMemsetAsync(ws->counter, 0, sizeof(unsigned long long), st);
  if (e == hipSuccess)
    e = launch_tile_count(P, params->fp64_alpha_threshold, lds, ws->counter,
                          st);
  unsigned long long h = 0;
  if (e == hipSuccess)
    e = hipMemcpyAsync(&h, ws->counter, sizeof h, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "bssn_mixed_tile_count");
  dim3 grd, blk;
  tile_grid(P, lds, grd, blk);
  *n_fp64 = (int64_t)h;
  *n_tiles = (int64_t)grd.x * grd.y * grd.z;
  g_err = "no error";
  return BSSN_OK;
}

}  // extern "C"
