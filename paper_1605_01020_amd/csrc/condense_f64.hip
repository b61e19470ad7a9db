// Condensation kernels, FP64 storage and FP64 MFMA (section 2.2.1, eq. LS).
// The batched (persistent) form; the one-element-per-workgroup kernels are
// in condense_f64_single.hip.
#include "condense_kernel.h"

namespace iedg {

hipError_t condense_launch_f64(const CondenseArgs<double>& a, const CondenseArgs<double>* segs, const QueueLaunch& q, int lw, int ct,
                               hipStream_t s) {
  if (!segs) return condense_single_f64(a, lw, ct, s);
  return dispatch_queue<double, 0>(s, segs, q.items, q.n_items, q.n_max, q.counter, q.n_wg);
}

int condense_queue_slots_f64(int n_max) { return queue_slots<double, 0>(n_max); }

}  // namespace iedg
