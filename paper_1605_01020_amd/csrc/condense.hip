// Element static condensation (section 2.2.1, eq. LS): host entry points,
// the batched plan, the sub-panel width table and the right-hand-side
// condensation kernel.  The condensation kernel itself is in
// condense_kernel.h, compiled once per precision.
#include <initializer_list>

#include "common.h"
#include "condense.h"

namespace iedg {

// ---- right-hand side condensation: w = L^{-1} P F, r = -L21 w ----------
// Position i of P A is physical row perm[i] of LU and of w.  Rows are taken
// four per wave at a time (wave_dot_rows, 16 loads in flight per lane);
// 64-row diagonal blocks of L are staged in LDS in the storage precision and
// solved by one wave.  LDS stays small so that several elements share a CU.
constexpr int RTHR = 256;

template <typename T>
__global__ __launch_bounds__(RTHR) void condense_rhs_kernel(int n, int t, const T* LU, const int32_t* perm,
                                                            const T* L21, const double* F, double* w,
                                                            double* r) {
  const int e = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr int RW = RTHR / 64;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* y = reinterpret_cast<double*>(smem_raw);      // n
  int* sp = reinterpret_cast<int*>(y + n);              // n
  T* blk = reinterpret_cast<T*>(sp + ((n + 3) & ~3));  // 64 x 65
  const T* L = LU + (size_t)e * n * n;
  const int32_t* p = perm + (size_t)e * n;
  const double* f = F + (size_t)e * n;
  for (int i = tid; i < n; i += RTHR) {
    sp[i] = p[i];
    y[i] = f[p[i]];
  }
  __syncthreads();
  for (int i0 = 0; i0 < n; i0 += 64) {
    const int i1 = min(i0 + 64, n), bw = i1 - i0;
    if (i0 > 0) {
      for (int i = i0 + 4 * wv; i < i1; i += 4 * RW) {
        const T* rows[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) rows[q] = L + (size_t)sp[min(i + q, i1 - 1)] * n;
        double s[4];
        wave_dot_rows<T, 4>(rows, y, i0, s);
        if (lane < 4 && i + lane < i1) {
          double v = s[0];
#pragma unroll
          for (int q = 1; q < 4; ++q) v = lane == q ? s[q] : v;
          y[i + lane] -= v;
        }
      }
    }
    for (int q = tid; q < 64 * 64; q += RTHR) {
      const int rr = q / 64, cc = q % 64;
      blk[rr * 65 + cc] = (rr < bw && cc < rr) ? L[(size_t)sp[i0 + rr] * n + i0 + cc] : T(0);
    }
    __syncthreads();
    if (wv == 0) {
      double yl = lane < bw ? y[i0 + lane] : 0.0;
      for (int k = 0; k < bw; ++k) {
        const double yk = __shfl(yl, k, kWave);
        if (lane > k) yl -= (double)blk[lane * 65 + k] * yk;
      }
      if (lane < bw) y[i0 + lane] = yl;
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += RTHR) w[(size_t)e * n + sp[i]] = y[i];
  const T* L2 = L21 + (size_t)e * t * n;
  for (int i = 4 * wv; i < t; i += 4 * RW) {
    const T* rows[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) rows[q] = L2 + (size_t)min(i + q, t - 1) * n;
    double s[4];
    wave_dot_rows<T, 4>(rows, y, n, s);
    if (lane < 4 && i + lane < t) {
      double v = s[0];
#pragma unroll
      for (int q = 1; q < 4; ++q) v = lane == q ? s[q] : v;
      r[(size_t)e * t + i + lane] = -v;
    }
  }
}

// The context's sub-panel width (field lw) or panel width (field ct) for
// (prec, n); with bf16_from_f32, BF16 without an entry of its own takes the
// FP32 entry; 0 (the kernel's default) when untuned.
static int tuned(iedg_context ctx, iedg_prec prec, int n, int iedg_context_s::LeafChoice::*field,
                 bool bf16_from_f32) {
  std::lock_guard<std::mutex> lock(ctx->leaf_mu);
  int fallback = 0;
  for (const auto& c : ctx->leaf) {
    if (c.n != n) continue;
    if (c.prec == (int)prec && c.*field) return c.*field;
    if (bf16_from_f32 && prec == IEDG_BF16 && c.prec == (int)IEDG_F32) fallback = c.*field;
  }
  return fallback;
}
static int leaf_width(iedg_context ctx, iedg_prec prec, int n) {
  return tuned(ctx, prec, n, &iedg_context_s::LeafChoice::lw, true);
}
// The panel width is not taken over from FP32: BF16 operands favour other
// widths (the operands are rounded on every fragment read).
static int panel_width(iedg_context ctx, iedg_prec prec, int n) {
  const int ct = tuned(ctx, prec, n, &iedg_context_s::LeafChoice::ct, false);
  return prec == IEDG_F64 ? 64 : ct;  // FP64 storage is built for 64 only
}

}  // namespace iedg

using namespace iedg;

extern "C" void iedg_batch_destroy(iedg_batch b);

// Every array of a condensation starts on a 16-byte boundary: the kernel
// moves FP32/FP64 data in 8- and 16-byte vectors (with n a multiple of 4 and
// t even, every element's block then starts aligned too).
static bool aligned16(std::initializer_list<const void*> ps) {
  for (const void* p : ps)
    if (reinterpret_cast<uintptr_t>(p) & 15) return false;
  return true;
}

extern "C" iedg_status iedg_condense(iedg_context ctx, int32_t n_elem, int32_t n_local, int32_t n_trace_elem,
                                     iedg_prec prec, const double* A, const double* B, const double* C,
                                     const double* D, const double* F, void* LU, int32_t* perm, void* U12,
                                     void* L21, double* w, void* Ke, double* r, hipStream_t stream) {
  if (!ctx) return IEDG_ERR_INVALID_ARG;
  if (n_elem < 0 || n_local <= 0 || n_trace_elem <= 0)
    return set_error(ctx, IEDG_ERR_INVALID_ARG, "condense: bad sizes E=%d n=%d t=%d", n_elem, n_local, n_trace_elem);
  if (n_elem == 0) return IEDG_OK;
  if (!A || !B || !C || !D || !LU || !perm || !U12 || !L21 || !Ke)
    return set_error(ctx, IEDG_ERR_INVALID_ARG, "condense: null pointer");
  if (F && (!w || !r)) return set_error(ctx, IEDG_ERR_INVALID_ARG, "condense: F given without w and r");
  if ((n_local & 3) || (n_trace_elem & 1))
    return set_error(ctx, IEDG_ERR_UNSUPPORTED, "condense: n must be a multiple of 4, t even");
  if (n_local > kCondenseMaxN || n_trace_elem > kCondenseMaxT)
    return set_error(ctx, IEDG_ERR_UNSUPPORTED, "condense: n=%d t=%d too large", n_local, n_trace_elem);
  if (!aligned16({A, B, C, D, F, LU, perm, U12, L21, w, Ke, r}))
    return set_error(ctx, IEDG_ERR_INVALID_ARG, "condense: arrays must be 16-byte aligned");
  hipError_t err;
  if (prec == IEDG_F64) {
    CondenseArgs<double> a{n_elem, n_local, n_trace_elem, A, B, C, D, F,
                           (double*)LU, (double*)U12, (double*)L21, (double*)Ke, perm, w, r, ctx->d_status, 0};
    err = condense_launch_f64(a, nullptr, QueueLaunch{}, leaf_width(ctx, prec, n_local), 64, stream);
  } else if (prec == IEDG_F32 || prec == IEDG_BF16) {
    CondenseArgs<float> a{n_elem, n_local, n_trace_elem, A, B, C, D, F,
                          (float*)LU, (float*)U12, (float*)L21, (float*)Ke, perm, w, r, ctx->d_status, 0};
    const int lw = leaf_width(ctx, prec, n_local), ct = panel_width(ctx, prec, n_local);
    err = prec == IEDG_F32 ? condense_launch_f32(a, nullptr, QueueLaunch{}, lw, ct, stream)
                           : condense_launch_bf16(a, nullptr, QueueLaunch{}, lw, ct, stream);
  } else {
    return set_error(ctx, IEDG_ERR_UNSUPPORTED, "condense: precision %d not built", (int)prec);
  }
  if (err != hipSuccess) return hip_check(ctx, err, "condense launch");
  return IEDG_OK;
}

extern "C" iedg_status iedg_condense_rhs(iedg_context ctx, int32_t n_elem, int32_t n_local, int32_t n_trace_elem,
                                         iedg_prec prec, const void* LU, const int32_t* perm, const void* L21,
                                         const double* F, double* w, double* r, hipStream_t stream) {
  if (!ctx) return IEDG_ERR_INVALID_ARG;
  if (n_elem < 0 || n_local <= 0 || n_trace_elem <= 0)
    return set_error(ctx, IEDG_ERR_INVALID_ARG, "condense_rhs: bad sizes");
  if (n_elem == 0) return IEDG_OK;
  if (!LU || !perm || !L21 || !F || !w || !r) return set_error(ctx, IEDG_ERR_INVALID_ARG, "condense_rhs: null pointer");
  const size_t smem0 = sizeof(double) * n_local + sizeof(int) * ((n_local + 3) & ~3);
  if (prec == IEDG_F64) {
    const size_t smem = smem0 + sizeof(double) * 64 * 65;
    auto k = condense_rhs_kernel<double>;
    IEDG_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
    hipLaunchKernelGGL(k, dim3(n_elem), dim3(RTHR), smem, stream, n_local, n_trace_elem, (const double*)LU, perm,
                       (const double*)L21, F, w, r);
  } else if (prec == IEDG_F32 || prec == IEDG_BF16) {
    const size_t smem = smem0 + sizeof(float) * 64 * 65;
    auto k = condense_rhs_kernel<float>;
    IEDG_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
    hipLaunchKernelGGL(k, dim3(n_elem), dim3(RTHR), smem, stream, n_local, n_trace_elem, (const float*)LU, perm,
                       (const float*)L21, F, w, r);
  } else {
    return set_error(ctx, IEDG_ERR_UNSUPPORTED, "condense_rhs: precision");
  }
  IEDG_LAUNCH_CHECK(ctx, "condense_rhs launch");
  return IEDG_OK;
}

// ---- batched condensation ---------------------------------------------------
struct iedg_batch_s {
  iedg_context ctx = nullptr;
  int n_max = 0, n_items = 0, n_wg = 0;
  iedg_prec prec = IEDG_F64;
  void* d_segs = nullptr;   // CondenseArgs<T>[n_seg]
  int2* d_items = nullptr;  // (segment, element) work list
  int* d_counter = nullptr; // queue position of the persistent launch
};

extern "C" iedg_status iedg_batch_create_sized(iedg_context ctx, int32_t n_seg, const iedg_condense_segment* segs,
                                               const int32_t* n_local, const int32_t* n_trace_elem, iedg_prec prec,
                                               iedg_batch* out) {
  if (!ctx || !out || n_seg <= 0 || !segs || !n_local || !n_trace_elem)
    return set_error(ctx, IEDG_ERR_INVALID_ARG, "batch_create: bad arguments");
  if (prec != IEDG_F64 && prec != IEDG_F32 && prec != IEDG_BF16)
    return set_error(ctx, IEDG_ERR_UNSUPPORTED, "batch_create: precision");
  *out = nullptr;
  std::vector<CondenseArgs<double>> a64;
  std::vector<CondenseArgs<float>> a32;
  int n_max = 0;
  for (int s = 0; s < n_seg; ++s) {
    const iedg_condense_segment& g = segs[s];
    const int n = n_local[s], t = n_trace_elem[s];
    if (n <= 0 || t <= 0) return set_error(ctx, IEDG_ERR_INVALID_ARG, "batch_create: segment %d sizes", s);
    if ((n & 3) || (t & 1) || n > kCondenseMaxN || t > kCondenseMaxT)
      return set_error(ctx, IEDG_ERR_UNSUPPORTED, "batch_create: segment %d n=%d t=%d", s, n, t);
    if (g.n_elem < 0 || (g.n_elem > 0 && (!g.A || !g.B || !g.C || !g.D || !g.LU || !g.perm || !g.U12 || !g.L21 || !g.Ke)))
      return set_error(ctx, IEDG_ERR_INVALID_ARG, "batch_create: segment %d incomplete", s);
    if (g.F && (!g.w || !g.r)) return set_error(ctx, IEDG_ERR_INVALID_ARG, "batch_create: segment %d F without w, r", s);
    if (!aligned16({g.A, g.B, g.C, g.D, g.F, g.LU, g.perm, g.U12, g.L21, g.w, g.Ke, g.r}))
      return set_error(ctx, IEDG_ERR_INVALID_ARG, "batch_create: segment %d arrays must be 16-byte aligned", s);
    // the width iedg_condense would use for this size now (context table or default)
    int lw = leaf_width(ctx, prec, n), ct = panel_width(ctx, prec, n);
    if (lw == 0) lw = default_leaf_width(prec == IEDG_F64 ? 8 : 4, n, t);
    if (ct == 0) ct = default_panel_width(prec == IEDG_F64 ? 8 : 4, n);
    if (g.n_elem > 0) n_max = std::max(n_max, n);
    a64.push_back(CondenseArgs<double>{g.n_elem, n, t, g.A, g.B, g.C, g.D, g.F, (double*)g.LU, (double*)g.U12,
                                       (double*)g.L21, (double*)g.Ke, g.perm, g.w, g.r, ctx->d_status, lw, ct});
    a32.push_back(CondenseArgs<float>{g.n_elem, n, t, g.A, g.B, g.C, g.D, g.F, (float*)g.LU, (float*)g.U12,
                                      (float*)g.L21, (float*)g.Ke, g.perm, g.w, g.r, ctx->d_status, lw, ct});
  }
  // Work list: size classes from the largest element down (the long items
  // start first, the persistent workgroups finish on short ones); within a
  // class the segments interleave, so that concurrently running workgroups
  // read different meshes' memory.
  std::vector<int> seg_order(n_seg);
  for (int s = 0; s < n_seg; ++s) seg_order[s] = s;
  std::stable_sort(seg_order.begin(), seg_order.end(), [&](int x, int y) {
    return n_local[x] != n_local[y] ? n_local[x] > n_local[y] : n_trace_elem[x] > n_trace_elem[y];
  });
  std::vector<int2> items;
  for (size_t c0 = 0; c0 < seg_order.size();) {
    size_t c1 = c0;
    int maxE = 0;
    while (c1 < seg_order.size() && n_local[seg_order[c1]] == n_local[seg_order[c0]] &&
           n_trace_elem[seg_order[c1]] == n_trace_elem[seg_order[c0]])
      maxE = std::max(maxE, (int)segs[seg_order[c1++]].n_elem);
    for (int e = 0; e < maxE; ++e)
      for (size_t k = c0; k < c1; ++k)
        if (e < segs[seg_order[k]].n_elem) items.push_back(make_int2(seg_order[k], e));
    c0 = c1;
  }
  auto* b = new iedg_batch_s();
  b->ctx = ctx;
  b->n_max = n_max;
  b->prec = prec;
  b->n_items = (int)items.size();
  if (!items.empty()) {
    const int slots = prec == IEDG_F64   ? condense_queue_slots_f64(n_max)
                      : prec == IEDG_F32 ? condense_queue_slots_f32(n_max)
                                         : condense_queue_slots_bf16(n_max);
    if (slots <= 0) {
      delete b;
      return set_error(ctx, IEDG_ERR_HIP, "batch_create: no occupancy for n=%d", n_max);
    }
    b->n_wg = std::min(slots, b->n_items);
  }
  const size_t seg_bytes = prec == IEDG_F64 ? a64.size() * sizeof(a64[0]) : a32.size() * sizeof(a32[0]);
  hipError_t e = hipMalloc(&b->d_segs, seg_bytes);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&b->d_items), std::max<size_t>(1, items.size()) * sizeof(int2));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&b->d_counter), sizeof(int));
  if (e == hipSuccess)
    e = hipMemcpy(b->d_segs, prec == IEDG_F64 ? (const void*)a64.data() : (const void*)a32.data(), seg_bytes,
                  hipMemcpyHostToDevice);
  if (e == hipSuccess && !items.empty())
    e = hipMemcpy(b->d_items, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    iedg_batch_destroy(b);
    return hip_check(ctx, e, "batch_create upload");
  }
  *out = b;
  return IEDG_OK;
}

extern "C" iedg_status iedg_batch_create(iedg_context ctx, int32_t n_seg, const iedg_condense_segment* segs,
                                         int32_t n_local, int32_t n_trace_elem, iedg_prec prec, iedg_batch* out) {
  if (!ctx || !out || n_seg <= 0 || !segs) return set_error(ctx, IEDG_ERR_INVALID_ARG, "batch_create: bad arguments");
  std::vector<int32_t> ns(n_seg, n_local), ts(n_seg, n_trace_elem);
  return iedg_batch_create_sized(ctx, n_seg, segs, ns.data(), ts.data(), prec, out);
}

extern "C" iedg_status iedg_condense_batched(iedg_context ctx, iedg_batch b, hipStream_t stream) {
  if (!ctx || !b) return IEDG_ERR_INVALID_ARG;
  if (b->n_items == 0) return IEDG_OK;
  const QueueLaunch q{b->d_items, b->n_items, b->n_max, b->n_wg, b->d_counter};
  hipError_t err;
  if (b->prec == IEDG_F64)
    err = condense_launch_f64(CondenseArgs<double>{}, (const CondenseArgs<double>*)b->d_segs, q, 0, 0, stream);
  else if (b->prec == IEDG_BF16)
    err = condense_launch_bf16(CondenseArgs<float>{}, (const CondenseArgs<float>*)b->d_segs, q, 0, 0, stream);
  else
    err = condense_launch_f32(CondenseArgs<float>{}, (const CondenseArgs<float>*)b->d_segs, q, 0, 0, stream);
  if (err != hipSuccess) return hip_check(ctx, err, "condense_batched launch");
  return IEDG_OK;
}

extern "C" void iedg_batch_destroy(iedg_batch b) {
  if (!b) return;
  if (b->d_segs) hipFree(b->d_segs);
  if (b->d_items) hipFree(b->d_items);
  if (b->d_counter) hipFree(b->d_counter);
  delete b;
}

extern "C" iedg_status iedg_set_leaf_width(iedg_context ctx, iedg_prec prec, int32_t n_local, int32_t leaf_width) {
  if (!ctx) return IEDG_ERR_INVALID_ARG;
  if (n_local <= 0 || (prec != IEDG_F64 && prec != IEDG_F32 && prec != IEDG_BF16) ||
      (leaf_width != 8 && leaf_width != 16))
    return set_error(ctx, IEDG_ERR_INVALID_ARG, "set_leaf_width: precision F64/F32/BF16, sub-panel width 8 or 16");
  std::lock_guard<std::mutex> lock(ctx->leaf_mu);
  for (auto& c : ctx->leaf)
    if (c.prec == (int)prec && c.n == n_local) {
      c.lw = leaf_width;
      return IEDG_OK;
    }
  ctx->leaf.push_back({(int)prec, n_local, leaf_width, 0});
  return IEDG_OK;
}

extern "C" iedg_status iedg_set_panel_width(iedg_context ctx, iedg_prec prec, int32_t n_local, int32_t panel_width) {
  if (!ctx) return IEDG_ERR_INVALID_ARG;
  if (n_local <= 0 || (prec != IEDG_F32 && prec != IEDG_BF16 && prec != IEDG_F64) ||
      (panel_width != 64 && panel_width != 128) || (prec == IEDG_F64 && panel_width != 64))
    return set_error(ctx, IEDG_ERR_INVALID_ARG, "set_panel_width: 64 or 128 (FP32/BF16 storage), 64 (FP64)");
  std::lock_guard<std::mutex> lock(ctx->leaf_mu);
  for (auto& c : ctx->leaf)
    if (c.prec == (int)prec && c.n == n_local) {
      c.ct = panel_width;
      return IEDG_OK;
    }
  ctx->leaf.push_back({(int)prec, n_local, 0, panel_width});
  return IEDG_OK;
}
