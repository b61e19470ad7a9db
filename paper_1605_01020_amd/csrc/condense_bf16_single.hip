// Condensation kernels, FP32 storage; GEMM updates on BF16 operands with FP32 accumulation (section 2.2.1, eq. LS):
// the one-element-per-workgroup launches of every size class, sub-panel
// width and panel width.
#include "condense_kernel.h"

namespace iedg {

hipError_t condense_single_bf16(const CondenseArgs<float>& a, int lw, int ct, hipStream_t s) {
  return dispatch_single<float, 1>(a, s, lw, ct);
}

}  // namespace iedg
