// bssn_batch_o8.hip -- order-8 instantiations of the batched stage kernels
// (many patches per launch).
#include "bssn_kernels.h"
#include "bssn_lds.h"
#include "bssn_stage.h"

namespace bssn {

hipError_t launch_batch_o8(const BatchLaunch& B, const Gauge& G, int stage,
                           int precision, hipStream_t st) {
  return launch_batch_t<8>(B, G, stage, precision, st);
}

}  // namespace bssn
