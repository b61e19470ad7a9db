// Shared declarations of the condensation translation units.
#pragma once

#include "common.h"

namespace iedg {

template <typename T>
struct CondenseArgs {
  int E, n, t;
  const double *A, *B, *C, *D, *F;
  T *LU, *U12, *L21, *Ke;
  int32_t* perm;
  double *w, *r;
  DeviceStatus* status;
  int lw;  // sub-panel width (8 or 16) of this segment in the batched form
  int ct;  // panel width (64 or 128) of this segment in the batched form
};

// The persistent batched form: n_wg workgroups take n_items (segment,
// element) items from a queue (counter: one device int, reset by the
// launch on the stream); LDS is sized for elements of up to n_max local dofs.
struct QueueLaunch {
  const int2* items;
  int n_items, n_max, n_wg;
  int* counter;
};

// One condensation launch.  segs == nullptr: elements 0 .. a.E-1 of `a`, one
// workgroup each, sub-panel width lw (8 or 16) and panel width ct (64, or
// 128 in FP32 storage), 0 for the untuned defaults.  Otherwise the batched
// form over segs as described by q (a, lw, ct unused).  Each is defined in
// the translation unit of its precision.
hipError_t condense_launch_f64(const CondenseArgs<double>& a, const CondenseArgs<double>* segs, const QueueLaunch& q,
                               int lw, int ct, hipStream_t s);
hipError_t condense_launch_f32(const CondenseArgs<float>& a, const CondenseArgs<float>* segs, const QueueLaunch& q,
                               int lw, int ct, hipStream_t s);
hipError_t condense_launch_bf16(const CondenseArgs<float>& a, const CondenseArgs<float>* segs, const QueueLaunch& q,
                                int lw, int ct, hipStream_t s);

// The one-element-per-workgroup launches, each precision in a translation
// unit of its own (condense_*_single.hip): lw, ct as above.
hipError_t condense_single_f64(const CondenseArgs<double>& a, int lw, int ct, hipStream_t s);
hipError_t condense_single_f32(const CondenseArgs<float>& a, int lw, int ct, hipStream_t s);
hipError_t condense_single_bf16(const CondenseArgs<float>& a, int lw, int ct, hipStream_t s);

// Persistent grid size of the batched form for LDS sized for n_max local
// dofs (0 on a HIP error), per precision.
int condense_queue_slots_f64(int n_max);
int condense_queue_slots_f32(int n_max);
int condense_queue_slots_bf16(int n_max);

// Untuned sub-panel width for elements of n local dofs and t trace dofs
// (512 threads, so q rows of A and C per thread): 16 where q x 16 register
// values stay within the register file without spilling (FP32 up to 4 rows
// per thread, FP64 up to 2), else 8.
inline int default_leaf_width(size_t elem_bytes, int n, int t) {
  const int qa = (n + 511) / 512, qc = (t + 511) / 512;
  const int q = (qa <= 1 && qc <= 1) ? 2 : (qa <= 3 && qc <= 1) ? 4 : 7;
  return (elem_bytes == 8 ? q <= 2 : q <= 4) ? 16 : 8;
}

// Untuned panel width: 128 columns for FP32 storage (FP32 or BF16
// operands) and elements of at least 1024 local dofs (measured: 128 wins at
// n = 1280 and 2500, loses at 540), else 64 (the only width FP64 storage is
// built for).
inline int default_panel_width(size_t elem_bytes, int n) {
  return elem_bytes == 4 && n >= 1024 ? 128 : 64;
}

// Largest n and t the kernel is built for (rows per thread: 5 of A, 2 of C).
constexpr int kCondenseMaxN = 5 * 512, kCondenseMaxT = 2 * 512;

}  // namespace iedg
