// Condensation kernels, FP64 storage and FP64 MFMA (section 2.2.1, eq. LS):
// the one-element-per-workgroup launches of every size class, sub-panel
// width and panel width.
#include "condense_kernel.h"

namespace iedg {

hipError_t condense_single_f64(const CondenseArgs<double>& a, int lw, int ct, hipStream_t s) {
  return dispatch_single<double, 0>(a, s, lw, ct);
}

}  // namespace iedg
