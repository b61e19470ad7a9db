// Internal helpers shared by the gfx950 kernels of libiedg.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "iedg.h"

namespace iedg {

constexpr int kWave = 64;

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Lane layouts of the 16x16x4 MFMA operations on gfx950 (measured on the
// device).  A operand: lane l holds A[l % 16][l / 16]; B operand: lane l
// holds B[l / 16][l % 16].  Accumulator element v of lane l sits at
// column l % 16 and row
//   FP64 (v_mfma_f64_16x16x4f64): l / 16 + 4 v
//   FP32 (v_mfma_f32_16x16x4f32): 4 (l / 16) + v
template <typename T> struct Mfma;

template <> struct Mfma<double> {
  typedef d4 acc_t;
  __device__ static inline acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  __device__ static inline acc_t mac(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

template <> struct Mfma<float> {
  typedef f4 acc_t;
  __device__ static inline acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
  __device__ static inline acc_t mac(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// Wave-wide sum (64 lanes) with a fixed butterfly order: deterministic.
__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Block-wide deterministic sum; `red` is LDS of at least blockDim/64 doubles.
// Every thread receives the result.
__device__ inline double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}

// Workgroup barrier for data exchanged through GLOBAL memory.  A plain
// __syncthreads() orders LDS traffic only: it waits for lgkmcnt, not for the
// wave's outstanding vector-memory stores, and another wave may then read a
// stale copy.  Drain this wave's vector-memory operations before the barrier
// and invalidate the CU's vector L1 after it.
__device__ inline void sync_global() {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  asm volatile("buffer_inv sc0" ::: "memory");
}

// Dot product of a contiguous row (len values) with an LDS vector by one
// wave; each lane keeps 8 loads in flight per round trip.
template <typename T>
__device__ inline double wave_dot(const T* row, const double* vec, int len) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int k0 = lane; k0 < len; k0 += 64 * 8) {
    T v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = k0 + 64 * j;
      v[j] = k < len ? row[k] : T(0);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = k0 + 64 * j;
      if (k < len) s += (double)v[j] * vec[k];
    }
  }
  return wave_sum(s);
}

// Dot products of R contiguous rows (len values each) with one LDS vector by
// one wave: 4 loads per row in flight per lane, all rows' loads issued
// together.  rows[r] must be a valid address even when unused (its result
// is ignored).  Every lane receives every sum.
template <typename T, int R>
__device__ inline void wave_dot_rows(const T* const (&rows)[R], const double* vec, int len, double (&out)[R]) {
  const int lane = threadIdx.x & 63;
  double s[R];
#pragma unroll
  for (int r = 0; r < R; ++r) s[r] = 0.0;
  for (int k0 = lane; k0 < len; k0 += 64 * 4) {
    T v[R][4];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = k0 + 64 * j;
        v[r][j] = rows[r][k < len ? k : 0];
      }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + 64 * j;
      if (k < len) {
        const double x = vec[k];
#pragma unroll
        for (int r = 0; r < R; ++r) s[r] += (double)v[r][j] * x;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) out[r] = wave_sum(s[r]);
}

// Device status word: the smallest failing index (element or block row)
// and its code in one 64-bit word, (index << 8) | -code, all ones when
// clear, so that one atomicMin keeps an index with its own code whatever
// the order in which failures arrive.
struct DeviceStatus {
  unsigned long long word;
};
constexpr unsigned long long kStatusClear = ~0ull;

__device__ inline void latch_status(DeviceStatus* st, int32_t code, int64_t index) {
  atomicMin(&st->word, (static_cast<unsigned long long>(index) << 8) | static_cast<unsigned long long>(-code & 0xff));
}

}  // namespace iedg

// ---- host-side context --------------------------------------------------
struct iedg_context_s {
  int device = 0;
  std::string last_error;
  iedg::DeviceStatus* d_status = nullptr;   // device
  iedg::DeviceStatus* h_status = nullptr;   // pinned host mirror
  double* h_scalars = nullptr;              // pinned host readback area
  // condensation sub-panel and panel widths by (precision, n), set by the
  // autotuner (0: the untuned default)
  struct LeafChoice { int prec, n, lw, ct; };
  std::vector<LeafChoice> leaf;
  std::mutex leaf_mu;
};

namespace iedg {

iedg_status set_error(iedg_context ctx, iedg_status s, const char* fmt, ...);
iedg_status hip_check(iedg_context ctx, hipError_t e, const char* what);
// Looks up this context's device address of the allocation-free residual's
// static scratch (once per device; the device must be current).
iedg_status residual_scratch_init(iedg_context ctx);

}  // namespace iedg

#define IEDG_HIP(ctx, call)                                              \
  do {                                                                   \
    hipError_t _e = (call);                                              \
    if (_e != hipSuccess) return iedg::hip_check((ctx), _e, #call);      \
  } while (0)

#define IEDG_LAUNCH_CHECK(ctx, what)                                     \
  do {                                                                   \
    hipError_t _e = hipGetLastError();                                   \
    if (_e != hipSuccess) return iedg::hip_check((ctx), _e, what);       \
  } while (0)
