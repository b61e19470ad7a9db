// Minimum discarded fill (MDF) ordering of the trace system's block rows on
// gfx950 (section 2.2.2, which applies the MDF reordering of Persson and
// Peraire at subdomain level to BILU(0)).
//
// Greedy elimination on the zero-fill pattern of K, entirely on the device
// in FP64.  Eliminating block row k adds -A_ik A_kk^{-1} A_kj to every pair
// (i, j) of live rows coupled to k; pairs in the pattern take the update
// (what BILU(0) does), pairs outside it are dropped.  The weight of k is the
// squared Frobenius norm of the dropped blocks.  Each step eliminates the
// live row of least weight (ties: smaller face id), updates the remaining
// matrix on the pattern and recomputes the weights of k's live neighbours,
// which are the only weights the step changes.
//
// Work per step, as launches over fixed grids whose surplus workgroups
// return at once (no host synchronisation inside the loop):
//   select  (1 workgroup): fold the previous step's weight partials, argmin
//   xk      X_q = A_kk^{-1} A_kj for the q-th live neighbour j of k
//   update  A_ij -= A_ik X_j for live neighbours i, j of k with (i, j) in P
//   invert  A_gg^{-1} for the live neighbours g of k (their pivots changed)
//   xg      X_gj = A_gg^{-1} A_gj for live neighbours j of each such g
//   fill    || A_ig X_gj ||_F^2 for the pairs (i, j) of g outside P
#include <algorithm>
#include <vector>

#include "blockops.h"
#include "common.h"
#include "mesh.h"

namespace iedg {

struct MdfCtl {
  int k;      // row eliminated in the current step
  int step;
};

struct MdfArgs {
  int b, n_rows, maxnb;
  const int32_t *row_ptr, *col_face, *row_face, *pos, *diag_slot;
  double* W;        // [nnzb][b][b] working copy of K (pattern slots)
  double* Ainv;     // [n_rows][b][b] inverse pivot blocks
  double* Xk;       // [maxnb][b][b]
  double* Xg;       // [n_rows or maxnb][maxnb][b][b]
  double* part;     // [n_rows or maxnb][maxnb][maxnb] weight partials
  double* w;        // [n_rows] weights
  int* live;        // [n_rows]
  MdfCtl* ctl;
  int32_t* order;   // [n_rows] faces in elimination order (device)
  DeviceStatus* status;
};

// Slot of block (r, face) in row r, or -1.
__device__ inline int find_slot(const MdfArgs& a, int r, int face) {
  for (int s = a.row_ptr[r]; s < a.row_ptr[r + 1]; ++s)
    if (a.col_face[s] == face) return s;
  return -1;
}

// The q-th live row coupled to row r (r itself excluded), in slot order, or
// -1; *slot receives its slot in row r.
__device__ inline int live_nb(const MdfArgs& a, int r, int q, int* slot) {
  int c = 0;
  for (int s = a.row_ptr[r]; s < a.row_ptr[r + 1]; ++s) {
    const int g = a.pos[a.col_face[s]];
    if (g == r || !a.live[g]) continue;
    if (c == q) {
      if (slot) *slot = s;
      return g;
    }
    ++c;
  }
  return -1;
}

// Squared Frobenius norm of A * B (b x b, column-major), every thread gets it.
__device__ double block_mm_sqnorm(int b, const double* A, const double* B, double* red) {
  typedef Mfma<double> MF;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nt = (b + 15) / 16, ntiles = nt * nt;
  double s = 0.0;
  for (int tI = wv; tI < ntiles; tI += STHR / 64) {
    const int i0 = (tI / nt) * 16, j0 = (tI % nt) * 16;
    const int ia = i0 + li, jb = j0 + li;
    MF::acc_t acc = MF::zero();
    for (int k0 = 0; k0 < b; k0 += 4) {
      const int k = k0 + lk;
      const double av = (ia < b && k < b) ? A[(size_t)k * b + ia] : 0.0;
      const double bv = (jb < b && k < b) ? B[(size_t)jb * b + k] : 0.0;
      acc = MF::mac(av, bv, acc);
    }
    // entries outside the block are exact zeros (zero operands)
#pragma unroll
    for (int v = 0; v < 4; ++v) s += acc[v] * acc[v];
  }
  return block_sum(s, red);
}

// Gauss-Jordan inverse of W's pivot block of row g into Ainv[g].
__device__ void invert_pivot(const MdfArgs& a, int g, unsigned char* smem_raw) {
  const int b = a.b;
  double* s = reinterpret_cast<double*>(smem_raw);               // b x (b+1)
  int* piv = reinterpret_cast<int*>(s + (size_t)b * (b + 1));    // b
  double* rv = reinterpret_cast<double*>(piv + 128);
  int* ri = reinterpret_cast<int*>(rv + 1);
  const double* D = a.W + (size_t)a.diag_slot[g] * b * b;
  for (int q = threadIdx.x; q < b * b; q += STHR) {
    const int c = q / b, r = q % b;
    s[r * (b + 1) + c] = D[q];
  }
  __syncthreads();
  const bool ok = gj_invert<double>(s, b, piv, rv, ri);
  if (!ok && threadIdx.x == 0) latch_status(a.status, IEDG_ERR_SINGULAR, a.row_face[g]);
  double* out = a.Ainv + (size_t)g * b * b;
  for (int q = threadIdx.x; q < b * b; q += STHR) {
    const int c = q / b, r = q % b;
    out[q] = s[r * (b + 1) + c];
  }
}

// Row whose weight group qg covers: every row (init) or the qg-th live
// neighbour of the eliminated row.
__device__ inline int group_row(const MdfArgs& a, int init, int qg) {
  if (init) return qg < a.n_rows ? qg : -1;
  return qg < a.maxnb ? live_nb(a, a.ctl->k, qg, nullptr) : -1;
}

__global__ __launch_bounds__(STHR) void mdf_invert_kernel(MdfArgs a, int init) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int g = group_row(a, init, blockIdx.x);
  if (g < 0) return;
  invert_pivot(a, g, smem_raw);
}

__global__ __launch_bounds__(STHR) void mdf_xk_kernel(MdfArgs a) {
  const int k = a.ctl->k;
  int skj;
  const int j = live_nb(a, k, blockIdx.x, &skj);
  if (j < 0) return;
  const size_t bb = (size_t)a.b * a.b;
  block_mm<double>(a.b, a.Ainv + (size_t)k * bb, a.W + (size_t)skj * bb, a.Xk + blockIdx.x * bb, 0);
}

__global__ __launch_bounds__(STHR) void mdf_update_kernel(MdfArgs a) {
  const int k = a.ctl->k;
  const int qi = blockIdx.x / a.maxnb, qj = blockIdx.x % a.maxnb;
  const int i = live_nb(a, k, qi, nullptr);
  const int j = live_nb(a, k, qj, nullptr);
  if (i < 0 || j < 0) return;
  const int sij = find_slot(a, i, a.row_face[j]);
  if (sij < 0) return;   // outside the pattern: dropped
  const int sik = find_slot(a, i, a.row_face[k]);
  const size_t bb = (size_t)a.b * a.b;
  block_mm<double>(a.b, a.W + (size_t)sik * bb, a.Xk + (size_t)qj * bb, a.W + (size_t)sij * bb, 1);
}

__global__ __launch_bounds__(STHR) void mdf_xg_kernel(MdfArgs a, int init) {
  const int qg = blockIdx.x / a.maxnb, qj = blockIdx.x % a.maxnb;
  const int g = group_row(a, init, qg);
  if (g < 0) return;
  int sgj;
  const int j = live_nb(a, g, qj, &sgj);
  if (j < 0) return;
  const size_t bb = (size_t)a.b * a.b;
  block_mm<double>(a.b, a.Ainv + (size_t)g * bb, a.W + (size_t)sgj * bb,
                   a.Xg + ((size_t)qg * a.maxnb + qj) * bb, 0);
}

__global__ __launch_bounds__(STHR) void mdf_fill_kernel(MdfArgs a, int init) {
  __shared__ double red[STHR / 64];
  const int m = a.maxnb;
  const int qg = blockIdx.x / (m * m), qi = (blockIdx.x / m) % m, qj = blockIdx.x % m;
  const int g = group_row(a, init, qg);
  double* out = a.part + blockIdx.x;
  int sgi = -1;
  const int i = g >= 0 ? live_nb(a, g, qi, &sgi) : -1;
  const int j = g >= 0 ? live_nb(a, g, qj, nullptr) : -1;
  if (i < 0 || j < 0 || i == j || find_slot(a, i, a.row_face[j]) >= 0) {
    if (threadIdx.x == 0) *out = 0.0;   // no fill dropped for this pair
    return;
  }
  const int sig = find_slot(a, i, a.row_face[g]);
  const size_t bb = (size_t)a.b * a.b;
  const double s = block_mm_sqnorm(a.b, a.W + (size_t)sig * bb, a.Xg + ((size_t)qg * m + qj) * bb, red);
  if (threadIdx.x == 0) *out = s;
}

// Initial weights: w[g] = sum of the partials of group g, fixed order.
__global__ void mdf_fold_all_kernel(MdfArgs a) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a.n_rows) return;
  const int mm = a.maxnb * a.maxnb;
  double s = 0.0;
  for (int q = 0; q < mm; ++q) s += a.part[(size_t)g * mm + q];
  a.w[g] = s;
}

// One workgroup: fold the previous step's partials into its neighbours'
// weights, then pick the live row of least (weight, face id).
constexpr int SEL_THR = 1024;
__global__ __launch_bounds__(SEL_THR) void mdf_select_kernel(MdfArgs a, int step) {
  __shared__ double bw[SEL_THR];
  __shared__ int bf[SEL_THR], br[SEL_THR];
  const int tid = threadIdx.x, m = a.maxnb;
  if (step > 0 && tid < m) {
    const int g = live_nb(a, a.ctl->k, tid, nullptr);
    if (g >= 0) {
      double s = 0.0;
      for (int q = 0; q < m * m; ++q) s += a.part[(size_t)tid * m * m + q];
      a.w[g] = s;
    }
  }
  __syncthreads();
  double best = 0.0;
  int bface = INT32_MAX, brow = -1;
  for (int r = tid; r < a.n_rows; r += SEL_THR) {
    if (!a.live[r]) continue;
    const double v = a.w[r];
    const int f = a.row_face[r];
    if (brow < 0 || v < best || (v == best && f < bface)) {
      best = v;
      bface = f;
      brow = r;
    }
  }
  bw[tid] = best;
  bf[tid] = bface;
  br[tid] = brow;
  __syncthreads();
  for (int off = SEL_THR / 2; off > 0; off >>= 1) {
    if (tid < off) {
      const int o = tid + off;
      const bool take = br[o] >= 0 && (br[tid] < 0 || bw[o] < bw[tid] || (bw[o] == bw[tid] && bf[o] < bf[tid]));
      if (take) {
        bw[tid] = bw[o];
        bf[tid] = bf[o];
        br[tid] = br[o];
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    const int k = br[0];
    a.ctl->k = k;
    a.ctl->step = step;
    a.order[step] = a.row_face[k];
    a.live[k] = 0;
  }
}

template <typename T>
__global__ void mdf_copy_kernel(const T* K, double* W, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) W[i] = (double)K[i];
}

__global__ void mdf_fill_int_kernel(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace iedg

using namespace iedg;

extern "C" iedg_status iedg_mdf_order(iedg_context ctx, iedg_mesh mesh, iedg_prec prec, const void* Kbsr,
                                      int32_t* order, hipStream_t stream) {
  if (!ctx || !mesh || !Kbsr || !order) return set_error(ctx, IEDG_ERR_INVALID_ARG, "mdf_order: null argument");
  if (prec != IEDG_F64 && prec != IEDG_F32 && prec != IEDG_BF16)
    return set_error(ctx, IEDG_ERR_INVALID_ARG, "mdf_order: precision %d", (int)prec);
  const int b = mesh->b, NF = mesh->n_face;
  int maxnb = 0;
  for (int i = 0; i < NF; ++i) maxnb = std::max(maxnb, mesh->row_ptr[i + 1] - mesh->row_ptr[i] - 1);
  maxnb = std::max(maxnb, 1);
  const size_t bb = (size_t)b * b, mm = (size_t)maxnb * maxnb;
  const size_t nW = (size_t)mesh->nnzb * bb, nA = (size_t)NF * bb, nXk = (size_t)maxnb * bb,
               nXg = (size_t)NF * maxnb * bb, nP = (size_t)NF * mm;
  // set-up call: FP64 working arrays, freed before returning
  double* buf = nullptr;
  int* ibuf = nullptr;
  const size_t total = nW + nA + nXk + nXg + nP + NF;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&buf), total * sizeof(double));
  if (e != hipSuccess) return set_error(ctx, IEDG_ERR_OOM, "mdf_order: %zu bytes", total * sizeof(double));
  e = hipMalloc(reinterpret_cast<void**>(&ibuf), (2 * (size_t)NF + 8) * sizeof(int));
  if (e != hipSuccess) {
    (void)hipFree(buf);
    return set_error(ctx, IEDG_ERR_OOM, "mdf_order: index arrays");
  }
  MdfArgs a;
  a.b = b;
  a.n_rows = NF;
  a.maxnb = maxnb;
  a.row_ptr = mesh->d_row_ptr;
  a.col_face = mesh->d_col_face;
  a.row_face = mesh->d_row_face;
  a.pos = mesh->d_pos;
  a.diag_slot = mesh->d_diag_slot;
  a.W = buf;
  a.Ainv = a.W + nW;
  a.Xk = a.Ainv + nA;
  a.Xg = a.Xk + nXk;
  a.part = a.Xg + nXg;
  a.w = a.part + nP;
  a.live = ibuf;
  a.order = ibuf + NF;
  a.ctl = reinterpret_cast<MdfCtl*>(ibuf + 2 * (size_t)NF);
  a.status = ctx->d_status;
  iedg_status st = IEDG_OK;
  auto fail = [&](hipError_t err, const char* what) {
    st = hip_check(ctx, err, what);
  };
  const unsigned g1 = (unsigned)((nW + 255) / 256);
  if (prec == IEDG_F64)
    hipLaunchKernelGGL(mdf_copy_kernel<double>, dim3(g1), dim3(256), 0, stream, (const double*)Kbsr, a.W,
                       (int64_t)nW);
  else
    hipLaunchKernelGGL(mdf_copy_kernel<float>, dim3(g1), dim3(256), 0, stream, (const float*)Kbsr, a.W,
                       (int64_t)nW);
  hipLaunchKernelGGL(mdf_fill_int_kernel, dim3((NF + 255) / 256), dim3(256), 0, stream, a.live, NF, 1);
  const size_t inv_smem = sizeof(double) * b * (b + 1) + sizeof(int) * 128 + 2 * sizeof(double);
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(mdf_invert_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)inv_smem);
  if (e != hipSuccess) fail(e, "mdf_order: LDS attribute");
  if (st == IEDG_OK) {
    // initial weights of every row
    hipLaunchKernelGGL(mdf_invert_kernel, dim3(NF), dim3(STHR), inv_smem, stream, a, 1);
    hipLaunchKernelGGL(mdf_xg_kernel, dim3((unsigned)(NF * maxnb)), dim3(STHR), 0, stream, a, 1);
    hipLaunchKernelGGL(mdf_fill_kernel, dim3((unsigned)(NF * mm)), dim3(STHR), 0, stream, a, 1);
    hipLaunchKernelGGL(mdf_fold_all_kernel, dim3((NF + 255) / 256), dim3(256), 0, stream, a);
    e = hipGetLastError();
    if (e != hipSuccess) fail(e, "mdf_order: initial weights");
  }
  for (int step = 0; step < NF && st == IEDG_OK; ++step) {
    hipLaunchKernelGGL(mdf_select_kernel, dim3(1), dim3(SEL_THR), 0, stream, a, step);
    if (step + 1 == NF) break;
    hipLaunchKernelGGL(mdf_xk_kernel, dim3(maxnb), dim3(STHR), 0, stream, a);
    hipLaunchKernelGGL(mdf_update_kernel, dim3((unsigned)mm), dim3(STHR), 0, stream, a);
    hipLaunchKernelGGL(mdf_invert_kernel, dim3(maxnb), dim3(STHR), inv_smem, stream, a, 0);
    hipLaunchKernelGGL(mdf_xg_kernel, dim3((unsigned)mm), dim3(STHR), 0, stream, a, 0);
    hipLaunchKernelGGL(mdf_fill_kernel, dim3((unsigned)(mm * maxnb)), dim3(STHR), 0, stream, a, 0);
    e = hipGetLastError();
    if (e != hipSuccess) fail(e, "mdf_order: step launch");
  }
  if (st == IEDG_OK) {
    e = hipMemcpyAsync(order, a.order, sizeof(int32_t) * NF, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) fail(e, "mdf_order: readback");
  }
  (void)hipStreamSynchronize(stream);
  (void)hipFree(buf);
  (void)hipFree(ibuf);
  return st;
}
