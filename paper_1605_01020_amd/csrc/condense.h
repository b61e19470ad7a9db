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
};

// One condensation launch (segs == nullptr: elements 0 .. a.E-1 of `a`;
// otherwise one workgroup per (segment, element) item).  lw: sub-panel
// width 8 or 16, 0 for the untuned default.  Each is defined in the
// translation unit of its precision.
hipError_t condense_launch_f64(const CondenseArgs<double>& a, const CondenseArgs<double>* segs, const int2* items,
                               int n_items, int lw, hipStream_t s);
hipError_t condense_launch_f32(const CondenseArgs<float>& a, const CondenseArgs<float>* segs, const int2* items,
                               int n_items, int lw, hipStream_t s);
hipError_t condense_launch_bf16(const CondenseArgs<float>& a, const CondenseArgs<float>* segs, const int2* items,
                                int n_items, int lw, hipStream_t s);

// Largest n and t the kernel is built for (rows per thread: 5 of A, 2 of C).
constexpr int kCondenseMaxN = 5 * 512, kCondenseMaxT = 2 * 512;

}  // namespace iedg
