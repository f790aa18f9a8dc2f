/*
 * bssn.h -- C ABI of the MI355X BSSN right-hand-side / RK4 library.
 *
 * The library evaluates the vacuum BSSN right-hand side of the Einstein
 * Toolkit paper (arXiv:1111.3344, section "Spacetime Curvature Evolution":
 * the BSSN definitions, the evolution equations for alpha, K, beta^i, B^i,
 * phi, gt_ij, At_ij, Gt^i with m = 1, the Ricci split R~_ij + R^phi_ij, 1+log
 * slicing and the Gamma-driver shift with the attenuation q(r)), discretised
 * with centred finite differences of 4th (or 8th) order, upwinded advection
 * for the partial_0 = partial_t - beta^j partial_j terms and Kreiss-Oliger
 * dissipation (same section, opening paragraph), and fuses it with the
 * stage update of a classical fourth-order Runge-Kutta method of lines
 * (the paper separates right-hand-side evaluation from time integration:
 * HydroBase's "Calculating the RHS in MoL" schedule group).
 *
 * General rules for every entry point:
 *  - Device pointers point to HBM allocated by the caller (e.g. PyTorch);
 *    host pointers are marked "host".  The library never frees, keeps or
 *    allocates caller memory in the RK4 path.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    All GPU work is enqueued asynchronously on it; kernel faults surface at
 *    the caller's next synchronisation.
 *  - Every call returns BSSN_OK or a negative BSSN_E* code and never throws.
 *    Arguments are validated before anything is enqueued; a call that fails
 *    validation enqueues nothing and leaves every output untouched.
 *    bssn_last_error() gives a message for the last failure of the calling
 *    host thread.
 *  - Not thread-safe per stream: calls on one stream from several host
 *    threads must be serialised by the caller.
 *
 * State layout (one "state buffer"): 25 float64 grid functions ("slots") in
 * structure-of-arrays order, element (slot, z, y, x) of the storage grid
 * (interior plus `ghost` layers on every face) at
 *      ptr[slot*sf + z*sz + y*sy + x],   0 <= x < n[0]+2*ghost, etc.
 * so ptr points to the ghost corner of slot 0 and x is contiguous.  For best
 * performance sy should be a multiple of 16 and ptr + ghost 128-byte aligned.
 * Slot order (the paper's evolved variables, phi-variant):
 *   0 phi | 1-6 gt_xx gt_xy gt_xz gt_yy gt_yz gt_zz | 7 K |
 *   8-13 At_xx At_xy At_xz At_yy At_yz At_zz | 14-16 Gt^x Gt^y Gt^z |
 *   17 alpha | 18-20 beta^x beta^y beta^z | 21-23 B^x B^y B^z |
 *   24 A (time-derivative variable of the lapse: zero source, advected and
 *        dissipated only).
 * Boundary handling: BSSN_BC_PERIODIC wraps stencil indices modulo n (ghost
 * memory is never read or written); BSSN_BC_STATIC reads the ghost layers as
 * fixed boundary data and writes interior points only, so the caller fills
 * the ghosts of every buffer that is read by a stencil (u_n and every stage
 * state) once, before the first stage.
 */
#ifndef BSSN_H
#define BSSN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BSSN_ABI_VERSION 2

enum {
  BSSN_OK = 0,
  BSSN_EINVAL = -1,      /* invalid argument (message in bssn_last_error)   */
  BSSN_ENOMEM = -2,      /* device or host allocation failed                */
  BSSN_EHIP = -3,        /* a HIP runtime call or launch failed             */
  BSSN_ESTALE = -4,      /* a batch plan no longer matches its buffers      */
  BSSN_EUNSUPPORTED = -5 /* valid request the library does not implement    */
};

enum { BSSN_FP64 = 0, BSSN_MIXED = 1 };            /* bssn_params.precision */
enum { BSSN_BC_STATIC = 0, BSSN_BC_PERIODIC = 1 }; /* bssn_grid.bc          */
enum { BSSN_NSLOT = 25 };

/* A uniform Cartesian patch (the paper's CoordBase description: which points
 * are evolved and which are set by boundary or symmetry conditions). */
typedef struct {
  int32_t n[3];       /* interior points along x, y, z; each >= 1            */
  int32_t ghost;      /* ghost layers per face: >= 3 (order 4), >= 5 (8)     */
  int64_t sy, sz, sf; /* element strides of a y-row, a z-plane, a slot;
                         sy >= n[0]+2g, sz >= sy*(n[1]+2g), sf >= sz*(n[2]+2g)
                         and 8*sf < 2^31 (one slot below 2 GiB)               */
  double origin[3];   /* coordinate of interior point (0,0,0)                */
  double h[3];        /* grid spacing, > 0                                    */
  int32_t bc;         /* BSSN_BC_STATIC or BSSN_BC_PERIODIC                  */
} bssn_grid;

/* Discretisation, precision and gauge parameters (gauge: the paper's 1+log
 * slicing f = lapse_f/alpha with K_0 = 0, Gamma-driver G = shift_G/alpha^2,
 * H = exp(4 phi), eta^i = eta q(r) B^i). */
typedef struct {
  int32_t fd_order;    /* 4 or 8                                              */
  int32_t precision;   /* BSSN_FP64, or BSSN_MIXED: stencils and algebra in
                          FP32 on differences taken from the centre value in
                          FP64, state and RK4 update in FP64, and tiles whose
                          minimum lapse is below fp64_alpha_threshold (near a
                          puncture) evaluated entirely in FP64               */
  double ko_eps;       /* Kreiss-Oliger strength, >= 0 (0.1)                 */
  double lapse_f;      /* 2.0                                                 */
  double shift_G;      /* 0.75                                                */
  double eta;          /* 0.5                                                 */
  double eta_R;        /* transition radius R of q(r) = min(1, R/r), r the
                          coordinate radius; <= 0 or infinite: q = 1          */
  int32_t lapse_static;/* 1: right-hand side of alpha forced to 0           */
  int32_t shift_static;/* 1: right-hand sides of beta and B forced to 0     */
  double fp64_alpha_threshold; /* BSSN_MIXED only (0.3)                       */
} bssn_params;

/* Version of this header the library was built from (BSSN_ABI_VERSION). */
int bssn_abi_version(void);

/* Kernel selection for bssn_rhs / rk4_stage (process-wide; results agree to
 * rounding, both are checked against the same reference):
 *   BSSN_PATH_AUTO    persistent kernel that stages every slot's stencil box
 *                     in LDS through buffer->LDS DMA, for static grids whose
 *                     layout gives 16-byte aligned rows (even strides and
 *                     ptr + ghost - R - 1 aligned, R = 3 or 5); the
 *                     direct-load kernel otherwise;
 *   BSSN_PATH_DIRECT  always the direct-load kernel (one thread per point,
 *                     stencil taps read through the caches).
 * Errors: BSSN_EINVAL for other values. */
enum { BSSN_PATH_AUTO = 0, BSSN_PATH_DIRECT = 1 };
int bssn_set_path(int path);

/* Message of the last failed call on this host thread; host memory owned by
 * the library, valid until the next call on this thread; never NULL. */
const char* bssn_last_error(void);

/* Right-hand side d_t u of every slot at every interior point.
 *   u    device, state buffer (read; ghosts read when bc is static)
 *   rhs  device, same layout as u; interior points written, ghosts untouched;
 *        must not alias u.
 * Errors: BSSN_EINVAL (bad grid/params/pointers, aliasing), BSSN_EHIP. */
int bssn_rhs(const bssn_grid* grid, const bssn_params* params,
             const double* u, double* rhs, void* stream);

/* Stage s (0..3) of classical RK4 (c = 0, 1/2, 1/2, 1; b = 1/6, 1/3, 1/3,
 * 1/6), with k = d_t u(u_s) evaluated in the same kernel:
 *   s = 0:  acc  = u_n + dt/6 k     u_out = u_n + dt/2 k     (u_s = u_n)
 *   s = 1:  acc += dt/3 k           u_out = u_n + dt/2 k
 *   s = 2:  acc += dt/3 k           u_out = u_n + dt   k
 *   s = 3:                          u_out = acc + dt/6 k     (= u_{n+1})
 * All buffers are device state buffers of the same layout; only interior
 * points are written.  u_s may alias u_n (stage 0); u_out must not alias
 * u_s or acc; acc must alias nothing; u_out may alias u_n only at stage 3.
 * One step is stages 0..3 with (u_s, u_out) = (u_n, a), (a, b), (b, a),
 * (a, u_n) for two scratch buffers a, b.
 * Errors: BSSN_EINVAL (incl. stage outside 0..3, non-finite dt), BSSN_EHIP. */
int rk4_stage(const bssn_grid* grid, const bssn_params* params, int stage,
              double dt, const double* u_n, const double* u_s, double* acc,
              double* u_out, void* stream);

/* Hamiltonian and momentum constraints (section "Other analysis modules":
 * H = R - K^i_j K^j_i + K^2, M_i = D_j K_i^j - D_i K, vacuum), evaluated in
 * the BSSN variables in FP64 with the grid's finite-difference order, plus
 * the conformal-connection constraint G^i = Gt^i - gt^jk Gt^i_jk.
 *   u        device state buffer
 *   H        device, 1 slot in the state layout (slot stride sf), or NULL
 *   M        device, 3 slots in the state layout, or NULL
 *   G        device, 3 slots in the state layout, or NULL
 *   centres  host, 3*ncent coordinates (ncent 0..16); interior points closer
 *            than r_exc to any centre are left out of the norms
 *   norms    device, 8 doubles: H_rms, H_max, |M|_rms, |M|_max, |G|_rms,
 *            |G|_max, N_used, N_nonfinite (rms = sqrt(sum/N_used) over used
 *            points with finite values; |M| the flat Euclidean norm).
 * The reduction order is fixed, so results are bitwise reproducible.  The
 * first call on a device allocates a small partial-sum workspace that lives
 * until the process ends.
 * Errors: BSSN_EINVAL, BSSN_ENOMEM, BSSN_EHIP. */
int bssn_constraints(const bssn_grid* grid, const bssn_params* params,
                     const double* u, double* H, double* M, double* G,
                     const double* centres, int ncent, double r_exc,
                     double* norms, void* stream);

/* bssn_constraints for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, validation, kernels and results (bitwise) as
 * bssn_constraints; the per-block partial norms go to a fixed device array
 * of the library (16 MiB per GPU, held until the process ends) instead of
 * a workspace the library allocates.  It calls no allocating routine.
 * Limit: grids of at most 262,144 constraint blocks (one block per 64 x 4
 * points of a plane, 32 x 8 when n_x <= 32; a 384^3 grid needs 221,184);
 * larger grids return BSSN_EINVAL before anything is enqueued.  Calls on
 * one GPU share the array: calls that overlap in time on one GPU (other
 * streams, other host threads) race and must be ordered by the caller.
 * Errors: BSSN_EINVAL, BSSN_EUNSUPPORTED, BSSN_EHIP. */
int bssn_constraints_noalloc(const bssn_grid* grid, const bssn_params* params,
                             const double* u, double* H, double* M, double* G,
                             const double* centres, int ncent, double r_exc,
                             double* norms, void* stream);

/* Initial conversion from the ADM variables to the BSSN state (section
 * "Spacetime Curvature Evolution", initial conditions): by the definitions
 *   phi = ln(det g)/12, gt_ij = e^{-4 phi} g_ij, K = g^ij K_ij,
 *   At_ij = e^{-4 phi}(K_ij - g_ij K/3), alpha, beta^i copied, B^i = 0,
 *   slot 24 (A) = 0,
 * at every storage point; Gt^i = gt^ij gt^kl Gt_jkl from centred differences
 * (order params->fd_order) of the converted metric at interior points, and on
 * the ghost layers, innermost first, by the cubic extrapolation
 *   X(p) = 4X(p-n) - 6X(p-2n) + 4X(p-3n) - X(p-4n)
 * along n, the outward normal of p's face, or the sum of the face normals at
 * an edge or corner (e.g. (1,1,0)).
 *   adm  device, 16 slots in the state layout (slot stride sf):
 *        g_xx g_xy g_xz g_yy g_yz g_zz, K_xx .. K_zz, alpha, beta^x..beta^z,
 *        at every storage point (det g > 0)
 *   u    device state buffer, written at every storage point
 * Needs n >= 4 on every axis (the extrapolation reaches 4 points inward) and
 * u != adm.  Enqueues 2 + ghost launches on `stream`.  Errors: BSSN_EINVAL,
 * BSSN_EUNSUPPORTED, BSSN_EHIP. */
int bssn_from_adm(const bssn_grid* grid, const bssn_params* params,
                  const double* adm, double* u, void* stream);

/* Puncture tracking (section "Analysis", object tracking): one first-order
 * Euler step of dx^i/dt = -beta^i per puncture, the shift of u interpolated
 * to the position by tricubic Lagrange interpolation on the 4 x 4 x 4
 * storage points around it (base node floor((x - x_0)/h) - 1 per axis, x_0
 * the coordinate of storage index 0; the block is shifted inward where it
 * would leave the storage grid, so positions near or beyond the edge are
 * extrapolated, never read outside).
 *   u       device state buffer
 *   pos     device, 3*npunct coordinates (x, y, z per puncture), updated in
 *           place: pos <- pos - dt beta(pos)
 *   npunct  1..65536
 * Enqueues one launch on `stream`.  Errors: BSSN_EINVAL, BSSN_EUNSUPPORTED,
 * BSSN_EHIP. */
int bssn_track_punctures(const bssn_grid* grid, const double* u, int npunct,
                         double* pos, double dt, void* stream);

/* Multipole coefficients (section "Analysis": the multipole module) of a
 * complex grid function u = re + i im on the coordinate sphere of radius
 * `radius` around `centre`:
 *   C^{lm} = integral of conj(sY_lm) u r^2 dOmega,  s = spin,
 * sY_lm Goldberg's spin-weighted harmonics (Condon-Shortley phase at
 * s = 0), the integral over ntheta Gauss-Legendre nodes in cos(theta) times
 * nphi uniform points in phi (exact for products of harmonics of one spin
 * up to the node counts), u at each point by tricubic Lagrange
 * interpolation on the 4 x 4 x 4 storage points around it (the block
 * shifted inward at the edge of the storage grid).
 *   re, im  device, one slot each in the grid's layout (element 0 of the
 *           storage grid); im may be NULL (a real field)
 *   centre  host, 3 values; radius > 0
 *   spin    -8..8;  lmax 0..16;  ntheta 1..1024;  nphi 1..4096
 *   work    device scratch of at least
 *           2 ntheta (nphi + 1) + 2 (lmax + 1)^2 min(64, ceil(ntheta nphi
 *           / 256)) doubles
 *   coeffs  device, 2 (lmax + 1)^2 doubles: (re, im) of C^{lm} at index
 *           l*l + l + m; zero for l < |spin|
 * Four launches on `stream`; the sums run in a fixed order (the result is
 * deterministic).  Errors: BSSN_EINVAL, BSSN_EUNSUPPORTED, BSSN_EHIP. */
int bssn_multipole(const bssn_grid* grid, const double* re, const double* im,
                   const double* centre, double radius, int spin, int lmax,
                   int ntheta, int nphi, double* work, double* coeffs,
                   void* stream);

/* The Weyl scalar Psi_4 (section "Analysis", gravitational waves: the
 * WeylScal4 module) at every interior point of a grid:
 *   Psi_4 = C_abcd n^a mb^b n^c mb^d
 * on the fiducial tetrad l, n = (u +- rhat)/sqrt2, m = (thetahat +
 * i phihat)/sqrt2 (u the slice's unit normal; the spatial triad from
 * phi~ = (-y, x, 0), r~ = (x, y, z) and theta~^i = sqrt(det g) g^ik eps_klm
 * phi~^l r~^m, coordinates relative to `centre`, orthonormalised with the
 * 3-metric by Gram-Schmidt in the order phi, r, theta), evaluated as the
 * paper's projection of the Riemann tensor from the 3+1 data (vacuum: the
 * Weyl tensor is the Riemann tensor).  The ADM metric and curvature come
 * from the state by inverting the BSSN definitions,
 * g_ij = e^{4 phi} gt_ij, K_ij = e^{4 phi}(At_ij + gt_ij K/3), and are
 * differentiated with the centred stencils of `fd_order` (mixed second
 * derivatives as products of first-derivative stencils); FP64 throughout.
 *   fd_order  4 or 8; the grid's ghost width must cover order/2 (the ABI's
 *             usual minimum, 3 or 5, is required)
 *   u         device state buffer (reads phi, gt_ij, K, At_ij at every
 *             point within order/2 of the interior)
 *   centre    host, 3 coordinates: the origin of the tetrad's x^i
 *   psi4      device, two slots in the grid's layout (element 0 of the
 *             storage grid; slot 1 at +sf): Re Psi_4 and Im Psi_4 at the
 *             interior points; ghost points are not written.  Must not
 *             overlap u.  The output can go straight to bssn_multipole
 *             (re = psi4, im = psi4 + sf) with spin -2.
 * Points on the tetrad's axis (x = y = 0 relative to the centre) have no
 * phi direction; their values are NaN.  One launch on `stream`.  Errors:
 * BSSN_EINVAL, BSSN_EUNSUPPORTED, BSSN_EHIP. */
int bssn_psi4(const bssn_grid* grid, int fd_order, const double* u,
              const double* centre, double* psi4, void* stream);

/* Radiative (Sommerfeld-type) outer boundary (section "Spacetime Curvature
 * Evolution", boundary conditions): the right-hand side on the ghost layers
 * of a static grid, which then become evolved boundary points.  Every
 * component X is taken to be an outgoing spherical wave X0 + u(r - v0 t)/r
 * near the boundary, giving the wave part
 *   S = -v0 (x^i d_i X)/r - v0 (X - X0)/r    (r = |x|, x the coordinates),
 * with second-order differences (centred, one-sided at the storage edge);
 * the rest of the source decays as r^-power and is carried outward from the
 * inward neighbour q = p - n (n the outward normal of p's face, edge or
 * corner): rhs(p) = S(p) + (r_q/r_p)^power (rhs(q) - S(q)), each layer from
 * the one inside it.  The recursion is evaluated in closed form (it
 * telescopes to the interior point p clamped into the interior box), so the
 * result equals the layer-by-layer one up to rounding.
 *   x0, v0  host, 25 values per slot: value at infinity, wave speed (>= 0)
 *   power   0..16 (2: the second-order decay the paper assumes)
 *   u       device state buffer
 *   rhs     device, the state layout; its interior holds the interior
 *           right-hand side (e.g. from bssn_rhs) and is read, not written;
 *           on return its ghost layers hold the boundary right-hand side
 * The grid must be BSSN_BC_STATIC with ghost >= 3, rhs != u, and the
 * coordinate origin must not be a ghost point.  Enqueues one launch on
 * `stream`.  Errors: BSSN_EINVAL, BSSN_EUNSUPPORTED, BSSN_EHIP. */
int bssn_radiative_rhs(const bssn_grid* grid, const double* x0,
                       const double* v0, int power, const double* u,
                       double* rhs, void* stream);

/* One RK4 stage of an evolution whose outer boundary is radiative (section
 * "Spacetime Curvature Evolution", boundary conditions: the boundary points'
 * right-hand side is integrated in time like the interior's).  The ghost
 * layers of the static grid are evolved points: every storage point of
 * u_out (and of acc) is written, the interior by the fused stage of
 * rk4_stage, the ghost layers by the radiative right-hand side of
 * bssn_radiative_rhs (x0, v0, power as there) put through the same stage
 * update:
 *   s = 0: acc = u_n + dt/6 k,  u_out = u_n + dt/2 k
 *   s = 1: acc = acc + dt/3 k,  u_out = u_n + dt/2 k
 *   s = 2: acc = acc + dt/3 k,  u_out = u_n + dt k
 *   s = 3:                      u_out = acc + dt/6 k
 * The boundary is carried outward from the interior right-hand side at the
 * outermost layer of interior points, which the interior stage leaves in k
 * (as it computes it: FP64, or in mixed precision the arithmetic of the
 * point's tile).
 *   stage, dt, u_n, u_s, acc, u_out  as rk4_stage (same aliasing rules)
 *   k   device work buffer in the state layout (25 slots), aliasing no other
 *       buffer; on return its outermost interior layer holds the interior
 *       right-hand side there, everything else in it is untouched
 * Needs a static grid whose coordinate origin is neither a ghost point nor
 * on the outermost interior layer (r = 0 there).  The launches of the
 * interior stage and one more on `stream`.  Errors: BSSN_EINVAL,
 * BSSN_EUNSUPPORTED, BSSN_EHIP. */
int rk4_stage_radiative(const bssn_grid* grid, const bssn_params* params,
                        int stage, double dt, const double* x0,
                        const double* v0, int power, const double* u_n,
                        const double* u_s, double* acc, double* u_out,
                        double* k, void* stream);

/* Number of tiles a BSSN_MIXED evaluation of u runs in FP64 (tiles whose
 * minimum lapse over their points is below params->fp64_alpha_threshold)
 * and the total number of tiles.  Tiles are those of the kernel a stage on
 * this grid runs under the current bssn_set_path: 16 x 4 x 4 points for the
 * LDS-pipelined kernel (static grids), single-plane 64 x 4 (n[0] > 32) or
 * 32 x 8 for the direct kernel.  Synchronous; n_fp64 and n_tiles are host
 * pointers. */
int bssn_mixed_tile_count(const bssn_grid* grid, const bssn_params* params,
                          const double* u, int64_t* n_fp64, int64_t* n_tiles,
                          void* stream);

/* ---- many uneven patches advanced together (the paper's mesh-refinement
 * components: many independent grids per level) ------------------------ */
typedef struct bssn_batch_plan bssn_batch_plan;

/* Build a plan for npatch independent static-boundary patches sharing one
 * bssn_params.  Per patch p (host arrays; the buffers are device pointers):
 *   grids[p]  host, the patch's grid (bc must be BSSN_BC_STATIC)
 *   u[p]      device state buffer holding u_n; receives u_{n+1} after each
 *             step
 *   a[p], b[p]  device scratch state buffers with the same ghosts as u[p]
 *   acc[p]    device scratch state buffer (ghosts unused)
 *   dt[p]     host, the patch's RK4 time step (finite, >= 0); patches of a
 *             refinement hierarchy step with their own level's dt
 * Every buffer must be device memory whose allocation holds the grid's 25
 * slots from the pointer on (checked with the allocation's address range).
 * autotune = 1 times every kernel tile (shape and z-block depth, see
 * batch_patches_describe) the layout allows, per patch size class, on the
 * given buffers, and keeps the fastest (tuning runs stage 0 only, which
 * writes a and acc: nothing visible once the plan is built); 0 uses the
 * default tile (the LDS-pipelined kernel where the layout allows it);
 * BSSN_BATCH_TILE(v) uses tile v (0..4, in the order listed under
 * batch_patches_describe) for every class.  The plan captures the four
 * stages of a step in a hipGraph, in one of two launch modes: persistent
 * (the work of each tile in use as one launch per RK4 stage over a device
 * work list; a persistent kernel for the LDS tile) or per patch (one launch
 * per patch and stage, the kernels batch_patches_unbatched uses).
 * autotune = 1 also times both modes (stage 0) and keeps the faster; the
 * flag BSSN_BATCH_PER_PATCH (alone or with BSSN_BATCH_TILE) selects the per
 * patch mode, otherwise the mode is persistent.  The plan stores copies of
 * the pointer arrays; the buffers must stay allocated while it lives.
 * Errors: BSSN_EINVAL (also for a forced tile the layout does not allow),
 * BSSN_ENOMEM, BSSN_EHIP. */
#define BSSN_BATCH_TILE(v) (0x100 | (v))
#define BSSN_BATCH_PER_PATCH 0x200
int batch_patches_plan(int npatch, const bssn_grid* grids,
                       const bssn_params* params, double* const* u,
                       double* const* a, double* const* b,
                       double* const* acc, const double* dt, int autotune,
                       bssn_batch_plan** plan, void* stream);

/* batch_patches_plan whose steps put u_{n+1} into u_new[p] instead of
 * u[p] (stage 3 writes u_new; u[p] keeps u_n): the form a stepper needs
 * that keeps earlier time levels, such as Berger-Oliger subcycling (the
 * paper's adaptive mesh refinement: a level's patches step together,
 * their ghost points filled between stages).  u_new[p] may equal u[p];
 * it must not alias a, b or acc.  Same validation and errors, plus
 * BSSN_EINVAL for a NULL u_new. */
int batch_patches_plan_out(int npatch, const bssn_grid* grids,
                           const bssn_params* params, double* const* u,
                           double* const* u_new, double* const* a,
                           double* const* b, double* const* acc,
                           const double* dt, int autotune,
                           bssn_batch_plan** plan, void* stream);

/* Advance every patch of the plan by nsteps RK4 steps (one graph launch per
 * step on `stream`).  Returns BSSN_ESTALE if the plan was invalidated. */
int batch_patches(bssn_batch_plan* plan, int nsteps, void* stream);

/* One RK4 stage (0..3) of every patch of the plan: the plan's launches of
 * that stage, replayed from their own graph on `stream`.  Stages 0..3 in
 * order make one step, as batch_patches does; between them the caller may
 * rewrite the ghost points of the next stage's input (u, a, b, a for stages
 * 0..3), as a refinement hierarchy does.  Errors: BSSN_EINVAL (stage out of
 * range, NULL plan), BSSN_ESTALE, BSSN_EHIP. */
int batch_patches_stage(bssn_batch_plan* plan, int stage, void* stream);

/* Same update without the persistent kernel or graph: one kernel launch per
 * patch and stage (the baseline the batched path is measured against). */
int batch_patches_unbatched(bssn_batch_plan* plan, int nsteps, void* stream);

/* Kernel tile chosen for each size class (classes in increasing extent;
 * a class holds the patches whose largest extent rounds up to the same
 * multiple of 16): writes up to max_classes entries of (class extent,
 * tile_x, tile_y, z-block depth) into host array out (4 int32 each).
 * The tiles: 0 (16, 4, 4) the LDS-pipelined kernel; 1 (64, 4, 1),
 * 2 (32, 8, 1), 3 (64, 4, 4), 4 (32, 8, 4) the direct kernel, one
 * workgroup per tile of one plane or of a 4-plane z-block.  Returns the number of classes (>= 0,
 * possibly more than max_classes) or an error code. */
int batch_patches_describe(const bssn_batch_plan* plan, int max_classes,
                           int32_t* out);

/* Launch mode of the plan's graph: 0 (persistent work lists) or
 * BSSN_BATCH_PER_PATCH; an error code for a NULL plan. */
int batch_patches_launch_mode(const bssn_batch_plan* plan);

/* Release the plan (its graph, work list and device copies). */
int batch_patches_destroy(bssn_batch_plan* plan);

/* ---- refinement hierarchy glue (the framework section's mesh refinement:
 * Berger-Oliger stepping with subcycling; fine-grid boundaries filled by
 * interpolation in space and time from the coarser level; the fine
 * solution put back into the coarse grid where they overlap) ----------- */
typedef struct bssn_amr_plan bssn_amr_plan;

typedef struct {
  int32_t level;      /* 0 = coarsest; level L has half the spacing of L-1 */
  bssn_grid grid;     /* the patch's grid (bc must be BSSN_BC_STATIC)       */
} bssn_amr_patch;

/* Plan the glue of a hierarchy of npatch (1..65536) cell-centred patches
 * (host array).  Every level up to the highest must hold a patch; the
 * patches of one level share its spacing and lattice (origins an integer
 * number of spacings apart), and a level's points lie a quarter coarse
 * spacing from the coarser level's points (fine cells split coarse cells
 * in eight).  For every ghost point of a patch on level L >= 1 the plan
 * takes, in this order: a copy from the first other level-L patch (in
 * list order) whose interior holds the point; else the tricubic
 * interpolation from the first level-(L-1) patch whose storage grid
 * (ghosts included) holds the 4 x 4 x 4 coarse block around it (nodes
 * floor(s) - 1 .. floor(s) + 2 per axis, s the point in coarse index
 * units; weights (-7, 105, 35, -5)/128 or their mirror).  A ghost point
 * covered by neither is an error (BSSN_EINVAL, naming the patch and
 * point).  Restriction: every interior point of a level-(L-1) patch whose
 * eight children lie in the interior of a level-L patch (the first in list
 * order) takes the tricubic midpoint interpolation of that patch's storage,
 * weights (-1, 9, 9, -1)/16 per axis.  Allocates the plan's lists on
 * the current device (32 B per copied ghost point and per restricted
 * point, 112 B per 8 x 8 x 8 box of prolonged ghost points; level-0 ghost
 * points inside another level-0 interior are planned as copies).  *out receives the plan.  Errors: BSSN_EINVAL, BSSN_EUNSUPPORTED,
 * BSSN_EHIP. */
int bssn_amr_plan_create(const bssn_amr_patch* patches, int npatch,
                         bssn_amr_plan** out);

/* Host array counts[3] <- for level `level` (0..nlevel-1): the ghost
 * points filled, how many of them are sibling copies, and the level-1
 * points restriction from this level writes (0 for level 0). */
int bssn_amr_plan_counts(const bssn_amr_plan* plan, int level,
                         int64_t* counts);

/* Fill the ghost points of every level-`level` patch, on `stream`, on the
 * plan's device.  Level 0 exchanges only: a level-0 ghost point inside
 * another level-0 patch's interior (the first in list order) takes its
 * value; the other level-0 ghosts (the physical boundary) are left alone,
 * and ntl, src_tabs, t_src and t are not read.
 *   u_tab     device array of npatch device state pointers (the layout of
 *             the patch's grid, pointing at element 0 of slot 0); the
 *             level-`level` entries are written (ghosts only) and read
 *             (interiors, for sibling copies); other entries are not read
 *   ntl       1..3 coarse time levels
 *   src_tabs  host array of ntl device arrays of npatch device state
 *             pointers: the coarse level's states at times t_src[l] (only
 *             the level-(level-1) entries are read)
 *   t_src     host, ntl distinct finite times; t the target time
 * Prolonged values are the Lagrange interpolation in time through the ntl
 * levels of the spatial interpolations.  One launch; no allocation.  The
 * pointer tables must stay valid until the launch has run.  Errors:
 * BSSN_EINVAL, BSSN_EHIP. */
int bssn_amr_fill_ghosts(const bssn_amr_plan* plan, int level,
                         double* const* u_tab, int ntl,
                         const double* const* const* src_tabs,
                         const double* t_src, double t, void* stream);

/* Restrict refined level `level` into level - 1, on `stream`:
 *   fine_tab    device array of npatch device state pointers (level-`level`
 *               entries read, ghosts included)
 *   coarse_tab  device array of npatch device state pointers (level-1
 *               entries: the covered interior points are written)
 * One launch; no allocation.  Errors: BSSN_EINVAL, BSSN_EHIP. */
int bssn_amr_restrict(const bssn_amr_plan* plan, int level,
                      const double* const* fine_tab, double* const* coarse_tab,
                      void* stream);

/* Release the plan (its device op lists); NULL is accepted. */
int bssn_amr_plan_destroy(bssn_amr_plan* plan);

#ifdef __cplusplus
}
#endif

#endif /* BSSN_H */
