// Condensation kernels, FP64 storage and FP64 MFMA (section 2.2.1, eq. LS).
#include "condense_kernel.h"

namespace iedg {

hipError_t condense_launch_f64(const CondenseArgs<double>& a, const CondenseArgs<double>* segs, const QueueLaunch& q, int lw, int ct,
                               hipStream_t s) {
  return dispatch_condense<double, 0>(a, s, lw, ct, segs, q.items, q.n_items, q.n_max, q.counter, q.n_wg);
}

int condense_queue_slots_f64(int n_max) { return queue_slots<double, 0>(n_max); }

}  // namespace iedg
