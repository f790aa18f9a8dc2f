// bssn_rhs_o4.hip -- order-4 instantiations of the stage kernels.
#include "bssn_kernels.h"
#include "bssn_lds.h"
#include "bssn_stage.h"

namespace bssn {

hipError_t launch_stage_o4(const Patch& P, const Gauge& G, int periodic,
                           int stage, int precision, int path, int nwg,
                           hipStream_t st, double* kout) {
  const bool lds = !periodic && path != PATH_DIRECT && lds_path_ok<4>(P);
  if (lds) return launch_stage_lds<4>(P, G, stage, precision, nwg, st, kout);
  if (kout) {
    // the direct kernels do not store the shell's right-hand side: the
    // shell kernel does, before the stage
    Patch S = P;
    S.out = kout;
    const hipError_t e = launch_shell_rhs_t<4>(S, G, st);
    if (e != hipSuccess) return e;
  }
  return periodic
             ? launch_stage_variant<4, true>(P, G, stage, precision, 0, st)
             : launch_stage_variant<4, false>(P, G, stage, precision, 0,
                                                   st);
}

hipError_t launch_patch_o4(const Patch& P, const Gauge& G, int stage,
                           int precision, int variant, int nwg,
                           hipStream_t st) {
  return launch_patch_t<4>(P, G, stage, precision, variant, nwg, st);
}

bool variant_ok_o4(const Patch& P, int variant) {
  return variant_ok_t<4>(P, variant);
}

}  // namespace bssn
