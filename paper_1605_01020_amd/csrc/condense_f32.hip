// Condensation kernels, FP32 storage and FP32 MFMA with FP32 accumulation (section 2.2.1, eq. LS).
#include "condense_kernel.h"

namespace iedg {

hipError_t condense_launch_f32(const CondenseArgs<float>& a, const CondenseArgs<float>* segs, const int2* items,
                               int n_items, int lw, hipStream_t s) {
  return dispatch_condense<float, 0>(a, s, lw, segs, items, n_items);
}

}  // namespace iedg
