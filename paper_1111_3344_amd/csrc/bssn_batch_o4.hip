// bssn_batch_o4.hip -- order-4 instantiations of the batched stage kernels
// (many patches per launch).
#include "bssn_kernels.h"
#include "bssn_lds.h"
#include "bssn_stage.h"

namespace bssn {

hipError_t launch_batch_o4(const BatchLaunch& B, const Gauge& G, int stage,
                           int precision, hipStream_t st) {
  return launch_batch_t<4>(B, G, stage, precision, st);
}

}  // namespace bssn
