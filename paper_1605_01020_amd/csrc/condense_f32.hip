// Condensation kernels, FP32 storage and FP32 MFMA with FP32 accumulation (section 2.2.1, eq. LS).
#include "condense_kernel.h"

namespace iedg {

hipError_t condense_launch_f32(const CondenseArgs<float>& a, const CondenseArgs<float>* segs, const QueueLaunch& q, int lw, int ct,
                               hipStream_t s) {
  return dispatch_condense<float, 0>(a, s, lw, ct, segs, q.items, q.n_items, q.n_max, q.counter, q.n_wg);
}

int condense_queue_slots_f32(int n_max) { return queue_slots<float, 0>(n_max); }

}  // namespace iedg
