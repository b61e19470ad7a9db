// Condensation kernels, FP32 storage and FP32 MFMA with FP32 accumulation (section 2.2.1, eq. LS):
// the one-element-per-workgroup launches of every size class, sub-panel
// width and panel width.
#include "condense_kernel.h"

namespace iedg {

hipError_t condense_single_f32(const CondenseArgs<float>& a, int lw, int ct, hipStream_t s) {
  return dispatch_single<float, 0>(a, s, lw, ct);
}

}  // namespace iedg
