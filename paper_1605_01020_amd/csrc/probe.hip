// Measured ceilings of the device, the second denominator of the roofline
// report beside the datasheet peaks: an MFMA loop per operand type (the
// instruction the condensation issues, eight independent accumulator chains
// per wave so that the matrix pipe never waits on a result) and a STREAM
// triad a = b + s c over HBM-resident arrays.
#include "common.h"

namespace iedg {
namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
constexpr int PROBE_THREADS = 512;
constexpr int CHAINS = 8;
constexpr int TRIAD_THREADS = 256, TRIAD_UNROLL = 4;

// KIND 0: FP64 16x16x4, 1: FP32 16x16x4, 2: BF16 16x16x16 (FP32 accumulation).
// Operands are ones, so every accumulator entry ends at K * iters exactly
// (K = 4, 4, 16): the per-thread sum written to sink checks the whole loop.
template <int KIND>
__global__ __launch_bounds__(PROBE_THREADS) void mfma_probe_kernel(int iters, double* sink) {
  double total = 0.0;
  if constexpr (KIND == 0) {
    d4 acc[CHAINS];
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) acc[c] = d4{0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < iters; ++i)
#pragma unroll
      for (int c = 0; c < CHAINS; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(1.0, 1.0, acc[c], 0, 0, 0);
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) total += (acc[c][0] + acc[c][1]) + (acc[c][2] + acc[c][3]);
  } else {
    f4 acc[CHAINS];
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) acc[c] = f4{0.f, 0.f, 0.f, 0.f};
    if constexpr (KIND == 1) {
      for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(1.f, 1.f, acc[c], 0, 0, 0);
    } else {
      const short one = 0x3F80;  // BF16 1.0
      const s4 a = s4{one, one, one, one};
      for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, a, acc[c], 0, 0, 0);
    }
#pragma unroll
    for (int c = 0; c < CHAINS; ++c)
      total += ((double)acc[c][0] + (double)acc[c][1]) + ((double)acc[c][2] + (double)acc[c][3]);
  }
  sink[(size_t)blockIdx.x * PROBE_THREADS + threadIdx.x] = total;
}

// a = b + s c on n2 pairs of doubles; each thread moves TRIAD_UNROLL pairs
// (coalesced: consecutive threads take consecutive pairs), all loads issued
// before the first store.
__global__ __launch_bounds__(TRIAD_THREADS) void triad_kernel(int64_t n2, const double2* __restrict__ b,
                                                              const double2* __restrict__ c, double s,
                                                              double2* __restrict__ a) {
  const int64_t base = (int64_t)blockIdx.x * (TRIAD_THREADS * TRIAD_UNROLL) + threadIdx.x;
  double2 x[TRIAD_UNROLL], y[TRIAD_UNROLL];
#pragma unroll
  for (int u = 0; u < TRIAD_UNROLL; ++u) {
    const int64_t i = base + (int64_t)u * TRIAD_THREADS;
    if (i < n2) {
      x[u] = b[i];
      y[u] = c[i];
    }
  }
#pragma unroll
  for (int u = 0; u < TRIAD_UNROLL; ++u) {
    const int64_t i = base + (int64_t)u * TRIAD_THREADS;
    if (i < n2) a[i] = double2{x[u].x + s * y[u].x, x[u].y + s * y[u].y};
  }
}

}  // namespace
}  // namespace iedg

using namespace iedg;

extern "C" {

iedg_status iedg_probe_mfma(iedg_context ctx, iedg_prec prec, int32_t n_wg, int32_t iters, double* sink,
                            double* flops, hipStream_t stream) {
  if (!ctx) return IEDG_ERR_INVALID_ARG;
  if (!sink || !flops || n_wg <= 0 || iters <= 0 || iters > (1 << 20))
    return set_error(ctx, IEDG_ERR_INVALID_ARG, "probe_mfma: bad arguments");
  const double k = prec == IEDG_BF16 ? 16.0 : 4.0;
  // per wave-instruction 2 * 16 * 16 * K flops; 8 waves, CHAINS chains
  *flops = 2.0 * 16.0 * 16.0 * k * (PROBE_THREADS / kWave) * CHAINS * (double)iters * (double)n_wg;
  if (prec == IEDG_F64)
    hipLaunchKernelGGL(mfma_probe_kernel<0>, dim3(n_wg), dim3(PROBE_THREADS), 0, stream, iters, sink);
  else if (prec == IEDG_F32)
    hipLaunchKernelGGL(mfma_probe_kernel<1>, dim3(n_wg), dim3(PROBE_THREADS), 0, stream, iters, sink);
  else if (prec == IEDG_BF16)
    hipLaunchKernelGGL(mfma_probe_kernel<2>, dim3(n_wg), dim3(PROBE_THREADS), 0, stream, iters, sink);
  else
    return set_error(ctx, IEDG_ERR_INVALID_ARG, "probe_mfma: unknown precision %d", (int)prec);
  IEDG_LAUNCH_CHECK(ctx, "probe_mfma launch");
  return IEDG_OK;
}

iedg_status iedg_probe_triad(iedg_context ctx, int64_t n, const double* b, const double* c, double s, double* a,
                             hipStream_t stream) {
  if (!ctx) return IEDG_ERR_INVALID_ARG;
  if (!a || !b || !c || n <= 0 || (n & 1) ||
      ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) | reinterpret_cast<uintptr_t>(c)) & 15))
    return set_error(ctx, IEDG_ERR_INVALID_ARG, "probe_triad: n must be even and positive, arrays 16-byte aligned");
  const int64_t n2 = n / 2, per = (int64_t)TRIAD_THREADS * TRIAD_UNROLL;
  const int64_t grid = (n2 + per - 1) / per;
  if (grid > INT32_MAX) return set_error(ctx, IEDG_ERR_UNSUPPORTED, "probe_triad: n too large");
  hipLaunchKernelGGL(triad_kernel, dim3((unsigned)grid), dim3(TRIAD_THREADS), 0, stream, n2,
                     reinterpret_cast<const double2*>(b), reinterpret_cast<const double2*>(c), s,
                     reinterpret_cast<double2*>(a));
  IEDG_LAUNCH_CHECK(ctx, "probe_triad launch");
  return IEDG_OK;
}

}  // extern "C"
