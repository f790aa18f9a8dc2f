// bssn_rhs_o8.hip -- order-8 instantiations of the stage kernels.
#include "bssn_kernels.h"
#include "bssn_stage.h"

namespace bssn {

hipError_t launch_stage_o8(const Patch& P, const Gauge& G, int periodic,
                           int stage, int precision, hipStream_t st) {
  return periodic
             ? launch_stage_variant<8, true>(P, G, stage, precision, st)
             : launch_stage_variant<8, false>(P, G, stage, precision, st);
}

}  // namespace bssn
