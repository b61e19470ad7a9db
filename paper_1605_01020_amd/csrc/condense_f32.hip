// Condensation kernels, FP32 storage and FP32 MFMA with FP32 accumulation (section 2.2.1, eq. LS).
// The batched (persistent) form; the one-element-per-workgroup kernels are
// in condense_f32_single.hip.
#include "condense_kernel.h"

namespace iedg {

hipError_t condense_launch_f32(const CondenseArgs<float>& a, const CondenseArgs<float>* segs, const QueueLaunch& q, int lw, int ct,
                               hipStream_t s) {
  if (!segs) return condense_single_f32(a, lw, ct, s);
  return dispatch_queue<float, 0>(s, segs, q.items, q.n_items, q.n_max, q.counter, q.n_wg);
}

int condense_queue_slots_f32(int n_max) { return queue_slots<float, 0>(n_max); }

}  // namespace iedg
