// Condensation kernels, FP32 storage; GEMM updates on BF16 operands with FP32 accumulation (section 2.2.1, eq. LS).
// The batched (persistent) form; the one-element-per-workgroup kernels are
// in condense_bf16_single.hip.
#include "condense_kernel.h"

namespace iedg {

hipError_t condense_launch_bf16(const CondenseArgs<float>& a, const CondenseArgs<float>* segs, const QueueLaunch& q, int lw, int ct,
                                hipStream_t s) {
  if (!segs) return condense_single_bf16(a, lw, ct, s);
  return dispatch_queue<float, 1>(s, segs, q.items, q.n_items, q.n_max, q.counter, q.n_wg);
}

int condense_queue_slots_bf16(int n_max) { return queue_slots<float, 1>(n_max); }

}  // namespace iedg
