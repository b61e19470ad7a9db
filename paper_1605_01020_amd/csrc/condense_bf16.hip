// Condensation kernels, FP32 storage; GEMM updates on BF16 operands with FP32 accumulation (section 2.2.1, eq. LS).
#include "condense_kernel.h"

namespace iedg {

hipError_t condense_launch_bf16(const CondenseArgs<float>& a, const CondenseArgs<float>* segs, const int2* items,
                                int n_items, int lw, hipStream_t s) {
  return dispatch_condense<float, 1>(a, s, lw, segs, items, n_items);
}

}  // namespace iedg
