// bssn_internal.h -- structures shared by the HIP kernels and the C-ABI glue
// (not part of the public ABI).
#pragma once
#include <stdint.h>

namespace bssn {

constexpr int NSLOT = 25;

// slot numbers (see include/bssn.h)
enum : int {
  PHI = 0, GXX = 1, GXY, GXZ, GYY, GYZ, GZZ, TRK = 7, AXX = 8, AXY, AXZ,
  AYY, AYZ, AZZ, GAMX = 14, GAMY, GAMZ, ALP = 17, BETX = 18, BETY, BETZ,
  BX = 21, BY, BZ, ADOT = 24
};

// What a stage kernel writes.
enum : int { ST_RHS = -1, ST_0 = 0, ST_1 = 1, ST_2 = 2, ST_3 = 3 };

// Which points a mixed-precision kernel takes: all, only tiles whose minimum
// lapse is >= the threshold (FP32 path), or only the others (FP64 path).
enum : int { TILE_ALL = 0, TILE_FP32 = 1, TILE_FP64 = 2 };

// One patch as the kernels see it.
struct Patch {
  const double* u_s;   // stage input (stencil reads)
  const double* u_n;   // step start (stages 0..2)
  double* acc;         // RK4 accumulator
  double* out;         // stage output (or the RHS for ST_RHS)
  int32_t n[3];
  int32_t ghost;
  int32_t sy, sz;      // element strides (fit 32 bits: a slot < 2 GB)
  int64_t sf;
  double origin[3];
  double h[3];
  double dt;
  // uniform inverse spacings, computed on the host so they stay in SGPRs:
  // 1/h_a, 1/h_a^2, and 1/(h_x h_y), 1/(h_x h_z), 1/(h_y h_z)
  double ih[3], ih2[3], ihm[3];
};

struct Gauge {
  double ko_eps, lapse_f, shift_G, eta, eta_R;  // eta_R <= 0: q = 1
  int32_t lapse_static, shift_static;
  double alpha_thr;
};

// Work items of the batched kernels.  LDS kernel: a run of tiles [tlo, thi)
// of one patch whose tile grid is ntx x nty x ntz (tiles numbered z fastest
// within an (x, y) column).  Direct kernel: the workgroup-shaped tile at
// (x0, y0) of a z-block of planes of one patch.
struct LdsItem {
  int32_t patch, tlo, thi, ntx, nty, ntz;
};
struct DirectItem {
  int32_t patch, x0, y0, z0;  // planes z0 .. z0 + depth - 1
};
// One LDS tile of one patch (the FP64 pass of mixed precision).
struct TileRef {
  int32_t patch, tile;
};

// A multiplier coprime to n near n times the golden ratio's fraction, so
// that i -> (i * perm) mod n is a permutation of 0 .. n - 1 that scatters
// neighbours (the tiles around a puncture) far apart.
inline int64_t tile_perm(int64_t n) {
  if (n <= 1) return 1;
  int64_t p = int64_t(double(n) * 0.6180339887498949);
  if (p < 1) p = 1;
  for (;; ++p) {
    int64_t a = p, b = n;
    while (b) {
      const int64_t r = a % b;
      a = b;
      b = r;
    }
    if (a == 1) return p;
  }
}

// Kernel variants a batch plan chooses between, per patch size class:
// the LDS-pipelined persistent kernel (16 x 4 x 4 tiles) and the direct-load
// kernel with 64 x 4 or 32 x 8 workgroups, each workgroup doing one plane
// or marching through a z-block of 4 planes.
enum : int {
  VAR_LDS = 0,
  VAR_D64 = 1,
  VAR_D32 = 2,
  VAR_D64Z4 = 3,
  VAR_D32Z4 = 4,
  NVAR = 5
};
constexpr int kLdsTile[3] = {16, 4, 4};  // LDS kernel tile (x, y, z)
// tile (x, y, z-block depth) of each variant
constexpr int kVarTile[NVAR][3] = {
    {16, 4, 4}, {64, 4, 1}, {32, 8, 1}, {64, 4, 4}, {32, 8, 4}};

}  // namespace bssn
