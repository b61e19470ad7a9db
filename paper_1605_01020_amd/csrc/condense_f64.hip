// Condensation kernels, FP64 storage and FP64 MFMA (section 2.2.1, eq. LS).
#include "condense_kernel.h"

namespace iedg {

hipError_t condense_launch_f64(const CondenseArgs<double>& a, const CondenseArgs<double>* segs, const int2* items,
                               int n_items, int lw, hipStream_t s) {
  return dispatch_condense<double, 0>(a, s, lw, segs, items, n_items);
}

}  // namespace iedg
