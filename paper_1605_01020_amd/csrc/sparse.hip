// Block-sparse trace system on gfx950: assembly of K and R (section 2.2.1,
// eq. LS), BILU(0) factorisation and its triangular sweeps, and the BSR
// matrix-vector product (section 2.2.2).  Blocks are b x b, column-major,
// stored in the row order of the mesh's ordering (see iedg.h).
#include "blockops.h"
#include "common.h"
#include "mesh.h"

namespace iedg {

// ---- assembly ----------------------------------------------------------
// One workgroup per BSR block: gather the (one or two) element sub-blocks
// Ke_e[a*b:(a+1)*b, c*b:(c+1)*b] (row-major t x t), sum in ascending element
// order and write the block transposed to column-major through LDS.
template <typename T>
__global__ __launch_bounds__(STHR) void assemble_k_kernel(int b, int t, const int32_t* asm_src, const T* Ke,
                                                          T* Kbsr) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* tile = reinterpret_cast<T*>(smem_raw);  // b x (b+1)
  const int64_t s = blockIdx.x;
  const int src0 = asm_src[2 * s], src1 = asm_src[2 * s + 1];
  const int bb = b * b;
  const size_t tt = (size_t)t * t;
  const T* p0 = Ke + (size_t)(src0 / 36) * tt + (size_t)((src0 % 36) / 6) * b * t + (size_t)(src0 % 6) * b;
  const T* p1 = src1 >= 0 ? Ke + (size_t)(src1 / 36) * tt + (size_t)((src1 % 36) / 6) * b * t + (size_t)(src1 % 6) * b
                          : nullptr;
  for (int i0 = threadIdx.x; i0 < bb; i0 += STHR * 8) {
    T v0[8], v1[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = i0 + STHR * j;
      const int rr = i / b, cc = i % b;
      v0[j] = i < bb ? p0[(size_t)rr * t + cc] : T(0);
      v1[j] = (p1 && i < bb) ? p1[(size_t)rr * t + cc] : T(0);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = i0 + STHR * j;
      if (i < bb) tile[(i / b) * (b + 1) + i % b] = p1 ? v0[j] + v1[j] : v0[j];
    }
  }
  __syncthreads();
  T* out = Kbsr + (size_t)s * bb;
  for (int i = threadIdx.x; i < bb; i += STHR) {
    const int cc = i / b, rr = i % b;
    out[i] = tile[rr * (b + 1) + cc];
  }
}

// R[f*b + l] = G[f*b + l] + sum over elements e (ascending) of r_e[a*b + l].
__global__ void assemble_r_kernel(int n_face, int b, int t, const int32_t* face_src, const double* r,
                                  const double* G, double* R) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n_face * b) return;
  const int f = (int)(i / b), l = (int)(i % b);
  double v = G ? G[i] : 0.0;
  if (r) {
    for (int k = 0; k < 2; ++k) {
      const int src = face_src[2 * f + k];
      if (src >= 0) v += r[(size_t)(src / 6) * t + (src % 6) * b + l];
    }
  }
  R[i] = v;
}

// ---- BSR products --------------------------------------------------------
// Threads form G = STHR / b groups of b lanes; lane rr of group g
// accumulates row rr over blocks g, g+G, ... of a slot range.  Reads of a
// column-major block by consecutive rr are contiguous.
template <typename T>
__device__ inline double block_row_sum(int b, const T* blocks, const int32_t* col_face, int s0, int s1,
                                       const double* x, int g, int G, int rr) {
  double acc = 0.0;
  if (g >= G) return 0.0;
  for (int s = s0 + g; s < s1; s += G) {
    const T* blk = blocks + (size_t)s * b * b + rr;
    const double* xs = x + (size_t)col_face[s] * b;
    // eight columns per round trip: eight block loads (contiguous across the
    // group's lanes) and eight vector loads in flight per lane
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = 0.0;
    int cc = 0;
    for (; cc + 8 <= b; cc += 8) {
      T m[8];
      double xv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        m[u] = blk[(size_t)(cc + u) * b];
        xv[u] = xs[cc + u];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] += (double)m[u] * xv[u];
    }
    for (; cc < b; ++cc) a[0] += (double)blk[(size_t)cc * b] * xs[cc];
    acc += ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  }
  return acc;
}

// Reduce the G group partials of row rr into red[rr]; fixed order.
__device__ inline void group_reduce(double* red, int b, int G, int g, int rr, double v) {
  if (g < G) red[g * b + rr] = v;
  __syncthreads();
  if (threadIdx.x < b) {
    double s = red[threadIdx.x];
    for (int k = 1; k < G; ++k) s += red[k * b + threadIdx.x];
    red[G * b + threadIdx.x] = s;
  }
  __syncthreads();
}

// y = K x  (mode 0)   or   y = rhs - K x  (mode 1)
template <typename T>
__global__ __launch_bounds__(STHR) void spmv_kernel(int b, const int32_t* row_face, const int32_t* row_ptr,
                                                    const int32_t* col_face, const T* K, const double* x,
                                                    const double* rhs, double* y, int mode, const int* skip) {
  __shared__ double red[STHR + 128];
  if (skip && *skip) return;
  const int i = blockIdx.x;
  const int G = STHR / b, g = threadIdx.x / b, rr = threadIdx.x % b;
  const double v = block_row_sum<T>(b, K, col_face, row_ptr[i], row_ptr[i + 1], x, g, G, rr);
  group_reduce(red, b, G, g, rr, v);
  if (threadIdx.x < b) {
    const size_t o = (size_t)row_face[i] * b + threadIdx.x;
    const double kx = red[G * b + threadIdx.x];
    y[o] = mode == 0 ? kx : rhs[o] - kx;
  }
}

// One level of the BILU(0) sweeps.  Forward (upper = 0): y_i = x_i - sum
// over lower slots L_ik y_k.  Backward (upper = 1): y_i = Uinv_i (y_i - sum
// over upper slots U_ij y_j).  x may equal y.
template <typename T>
__global__ __launch_bounds__(STHR) void sweep_kernel(int b, const int32_t* rows, const int32_t* row_face,
                                                     const int32_t* row_ptr, const int32_t* diag_slot,
                                                     const int32_t* col_face, const T* M, const double* x,
                                                     double* y, int upper, const int* skip) {
  __shared__ double red[STHR + 128];
  if (skip && *skip) return;
  const int i = rows[blockIdx.x];
  const int G = STHR / b, g = threadIdx.x / b, rr = threadIdx.x % b;
  const int ds = diag_slot[i];
  const int s0 = upper ? ds + 1 : row_ptr[i];
  const int s1 = upper ? row_ptr[i + 1] : ds;
  const double v = block_row_sum<T>(b, M, col_face, s0, s1, y, g, G, rr);
  group_reduce(red, b, G, g, rr, v);
  const size_t o = (size_t)row_face[i] * b;
  if (!upper) {
    if (threadIdx.x < b) y[o + threadIdx.x] = x[o + threadIdx.x] - red[G * b + threadIdx.x];
    return;
  }
  // s = x_i - sum  ->  red[0:b]; then y_i = Uinv s
  __shared__ double svec[128];
  if (threadIdx.x < b) svec[threadIdx.x] = x[o + threadIdx.x] - red[G * b + threadIdx.x];
  __syncthreads();
  double acc = 0.0;
  if (g < G) {
    const T* blk = M + (size_t)ds * b * b + rr;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    int cc = g;
    for (; cc + 3 * G < b; cc += 4 * G) {
      T m[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) m[u] = blk[(size_t)(cc + u * G) * b];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] += (double)m[u] * svec[cc + u * G];
    }
    for (; cc < b; cc += G) a[0] += (double)blk[(size_t)cc * b] * svec[cc];
    acc = (a[0] + a[1]) + (a[2] + a[3]);
  }
  group_reduce(red, b, G, g, rr, acc);
  if (threadIdx.x < b) y[o + threadIdx.x] = red[G * b + threadIdx.x];
}

// ---- BILU(0) factorisation ------------------------------------------------
// One level of BILU(0): one workgroup per block row i of the level.
template <typename T>
__global__ __launch_bounds__(STHR) void ilu0_level_kernel(int b, const int32_t* rows, const int32_t* diag_slot,
                                                          const int32_t* lptr, const int32_t* lslot,
                                                          const int32_t* uptr, const int32_t* upd, T* M,
                                                          DeviceStatus* status) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* a = reinterpret_cast<T*>(smem_raw);                        // b x (b+1)
  int* piv = reinterpret_cast<int*>(a + (size_t)b * (b + 1));   // b
  double* rv = reinterpret_cast<double*>(piv + 128);            // 1
  int* ri = reinterpret_cast<int*>(rv + 1);                     // 1
  const int i = rows[blockIdx.x];
  const size_t bb = (size_t)b * b;
  for (int l = lptr[i]; l < lptr[i + 1]; ++l) {
    const int sik = lslot[2 * l], dk = lslot[2 * l + 1];
    // L_ik = A_ik * Uinv_k
    block_mm<T>(b, M + sik * bb, M + dk * bb, M + sik * bb, 0);
    sync_global();
    for (int u = uptr[l]; u < uptr[l + 1]; ++u) {
      const int skj = upd[2 * u], sij = upd[2 * u + 1];
      block_mm<T>(b, M + sik * bb, M + skj * bb, M + sij * bb, 1);
    }
    sync_global();
  }
  // pivot block: invert in place
  T* D = M + diag_slot[i] * bb;
  for (int q = threadIdx.x; q < b * b; q += STHR) {
    const int c = q / b, r = q % b;
    a[r * (b + 1) + c] = D[q];
  }
  __syncthreads();
  const bool ok = gj_invert<T>(a, b, piv, rv, ri);
  if (!ok && threadIdx.x == 0) latch_status(status, IEDG_ERR_SINGULAR, i);
  for (int q = threadIdx.x; q < b * b; q += STHR) {
    const int c = q / b, r = q % b;
    D[q] = a[r * (b + 1) + c];
  }
}

// One level of BILU(0) with both operands of every block product staged in
// LDS (b x b blocks, column-major, stride b + 1): sX holds A_ik and then
// L_ik = A_ik U_kk^{-1}; sB holds the right operand (U_kk^{-1}, then each
// U_kj).  Products run on MFMA with 16 x 16 tiles dealt round-robin to the
// four waves; A_ij -= L_ik U_kj is applied tile by tile to global memory.
// Copy up to two b x b blocks from global to LDS (stride b + 1), 8 loads in
// flight per thread per block.
template <typename T>
__device__ inline void lds_block_load2(const T* g0, T* s0, const T* g1, T* s1, int b) {
  const int ls = b + 1, bb = b * b;
  for (int q0 = threadIdx.x; q0 < bb; q0 += STHR * 8) {
    T v0[8], v1[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int q = q0 + STHR * j;
      v0[j] = q < bb ? g0[q] : T(0);
      v1[j] = (g1 && q < bb) ? g1[q] : T(0);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int q = q0 + STHR * j;
      if (q < bb) {
        const int c = q / b, r = q % b;
        s0[c * ls + r] = v0[j];
        if (g1) s1[c * ls + r] = v1[j];
      }
    }
  }
}

template <typename T>
__device__ inline void lds_block_mm(int b, const T* sA, const T* sB, typename Mfma<T>::acc_t (&acc)[16]) {
  typedef Mfma<T> MF;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int nt = (b + 15) / 16, ntiles = nt * nt, ls = b + 1;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    acc[q] = MF::zero();
    const int tI = wv + 4 * q;
    if (tI < ntiles) {
      const int i0 = (tI / nt) * 16, j0 = (tI % nt) * 16;
      const int ia = i0 + li, jb = j0 + li;
      for (int k0 = 0; k0 < b; k0 += 4) {
        const int k = k0 + lg;
        const T av = (ia < b && k < b) ? sA[k * ls + ia] : T(0);
        const T bv = (jb < b && k < b) ? sB[jb * ls + k] : T(0);
        acc[q] = MF::mac(av, bv, acc[q]);
      }
    }
  }
}

// STAGE_C: the block being updated is staged in LDS too (three b x b buffers);
// otherwise (large b) the update is applied to it in global memory in the
// accumulator layout and two buffers suffice.
template <typename T, bool STAGE_C>
__global__ __launch_bounds__(STHR) void ilu0_level_lds_kernel(int b, const int32_t* rows, const int32_t* diag_slot,
                                                              const int32_t* lptr, const int32_t* lslot,
                                                              const int32_t* uptr, const int32_t* upd, T* M,
                                                              DeviceStatus* status) {
  typedef Mfma<T> MF;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int ls = b + 1;
  T* sX = reinterpret_cast<T*>(smem_raw);   // b x ls: A_ik, then L_ik
  T* sB = sX + (size_t)b * ls;              // b x ls: right operand
  T* sC = sB + (size_t)b * ls;              // b x ls: block being updated (STAGE_C)
  int* piv = reinterpret_cast<int*>(STAGE_C ? sC + (size_t)b * ls : sC);
  double* rv = reinterpret_cast<double*>(piv + 128);
  int* ri = reinterpret_cast<int*>(rv + 1);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, li = lane & 15;
  const int nt = (b + 15) / 16, ntiles = nt * nt;
  const int i = rows[blockIdx.x];
  const size_t bb = (size_t)b * b;
  typename MF::acc_t acc[16];
  for (int l = lptr[i]; l < lptr[i + 1]; ++l) {
    const int sik = lslot[2 * l], dk = lslot[2 * l + 1];
    lds_block_load2<T>(M + sik * bb, sX, M + dk * bb, sB, b);
    __syncthreads();
    lds_block_mm<T>(b, sX, sB, acc);
    __syncthreads();
    // L_ik into sX (LDS), then to M[sik] from LDS (coalesced)
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int tI = wv + 4 * q;
      if (tI < ntiles) {
        const int i0 = (tI / nt) * 16, j0 = (tI % nt) * 16;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = i0 + MF::row(lane, v), c = j0 + li;
          if (r < b && c < b) sX[c * ls + r] = acc[q][v];
        }
      }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < (int)bb; q += STHR) M[sik * bb + q] = sX[(q / b) * ls + q % b];
    for (int u = uptr[l]; u < uptr[l + 1]; ++u) {
      const int skj = upd[2 * u], sij = upd[2 * u + 1];
      T* C = M + sij * bb;
      if constexpr (STAGE_C) {
        lds_block_load2<T>(M + skj * bb, sB, C, sC, b);
      } else {
        lds_block_load2<T>(M + skj * bb, sB, nullptr, nullptr, b);
      }
      __syncthreads();
      lds_block_mm<T>(b, sX, sB, acc);
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int tI = wv + 4 * q;
        if (tI < ntiles) {
          const int i0 = (tI / nt) * 16, j0 = (tI % nt) * 16;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = i0 + MF::row(lane, v), c = j0 + li;
            if (r < b && c < b) {
              if constexpr (STAGE_C)
                sC[c * ls + r] -= acc[q][v];
              else
                C[(size_t)c * b + r] -= acc[q][v];
            }
          }
        }
      }
      if constexpr (STAGE_C) {
        __syncthreads();
        for (int q = threadIdx.x; q < (int)bb; q += STHR) C[q] = sC[(q / b) * ls + q % b];
        __syncthreads();
      } else {
        sync_global();  // sB is reloaded next; C may be updated again
      }
    }
    sync_global();
  }
  // pivot block: invert in place (row-major staging in sX)
  T* Dg = M + diag_slot[i] * bb;
  T* sD = STAGE_C ? sC : sB;
  lds_block_load2<T>(Dg, sD, nullptr, nullptr, b);
  __syncthreads();
  for (int q = threadIdx.x; q < (int)bb; q += STHR) {
    const int c = q / b, r = q % b;
    sX[r * ls + c] = sD[c * ls + r];
  }
  __syncthreads();
  const bool ok = gj_invert<T>(sX, b, piv, rv, ri);
  if (!ok && threadIdx.x == 0) latch_status(status, IEDG_ERR_SINGULAR, i);
  for (int q = threadIdx.x; q < (int)bb; q += STHR) {
    const int c = q / b, r = q % b;
    Dg[q] = sX[r * ls + c];
  }
}

template <typename T>
static size_t elem_size() { return sizeof(T); }

static size_t prec_size(iedg_prec p) { return p == IEDG_F64 ? sizeof(double) : sizeof(float); }

}  // namespace iedg

using namespace iedg;

namespace iedg {

iedg_status spmv_launch(iedg_context ctx, iedg_mesh m, iedg_prec kprec, const void* K, const double* x,
                        const double* rhs, double* y, int mode, hipStream_t stream, const int* skip) {
  if (kprec == IEDG_F64)
    hipLaunchKernelGGL(spmv_kernel<double>, dim3(m->n_face), dim3(STHR), 0, stream, m->b, m->d_row_face,
                       m->d_row_ptr, m->d_col_face, (const double*)K, x, rhs, y, mode, skip);
  else
    hipLaunchKernelGGL(spmv_kernel<float>, dim3(m->n_face), dim3(STHR), 0, stream, m->b, m->d_row_face,
                       m->d_row_ptr, m->d_col_face, (const float*)K, x, rhs, y, mode, skip);
  IEDG_LAUNCH_CHECK(ctx, "spmv launch");
  return IEDG_OK;
}

// y = M^{-1} x : forward sweep over levels, then backward sweep in reverse.
iedg_status ilu0_apply_launch(iedg_context ctx, iedg_mesh m, iedg_prec mprec, const void* M, const double* x,
                              double* y, hipStream_t stream, const int* skip) {
  for (int dir = 0; dir < 2; ++dir) {
    for (int li = 0; li < m->n_levels; ++li) {
      const int l = dir == 0 ? li : m->n_levels - 1 - li;
      const int r0 = m->level_ptr[l], cnt = m->level_ptr[l + 1] - r0;
      const double* src = dir == 0 ? x : y;
      if (mprec == IEDG_F64)
        hipLaunchKernelGGL(sweep_kernel<double>, dim3(cnt), dim3(STHR), 0, stream, m->b, m->d_level_rows + r0,
                           m->d_row_face, m->d_row_ptr, m->d_diag_slot, m->d_col_face, (const double*)M, src, y,
                           dir, skip);
      else
        hipLaunchKernelGGL(sweep_kernel<float>, dim3(cnt), dim3(STHR), 0, stream, m->b, m->d_level_rows + r0,
                           m->d_row_face, m->d_row_ptr, m->d_diag_slot, m->d_col_face, (const float*)M, src, y,
                           dir, skip);
    }
  }
  IEDG_LAUNCH_CHECK(ctx, "ilu0 sweep launch");
  return IEDG_OK;
}

}  // namespace iedg

extern "C" {

iedg_status iedg_assemble(iedg_context ctx, iedg_mesh m, iedg_prec prec, const void* Ke, const double* r,
                          const double* G, void* Kbsr, double* R, hipStream_t stream) {
  if (!ctx || !m) return IEDG_ERR_INVALID_ARG;
  if ((Ke == nullptr) != (Kbsr == nullptr)) return set_error(ctx, IEDG_ERR_INVALID_ARG, "assemble: Ke and Kbsr go together");
  if ((r || G) && !R) return set_error(ctx, IEDG_ERR_INVALID_ARG, "assemble: R missing");
  if (prec != IEDG_F64 && prec != IEDG_F32 && prec != IEDG_BF16)
    return set_error(ctx, IEDG_ERR_INVALID_ARG, "assemble: precision");
  if (Ke) {
    const size_t smem = prec_size(prec) * m->b * (m->b + 1);
    if (prec == IEDG_F64) {
      auto k = assemble_k_kernel<double>;
      IEDG_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
      hipLaunchKernelGGL(k, dim3(m->nnzb), dim3(STHR), smem, stream, m->b, m->t, m->d_asm_src, (const double*)Ke,
                         (double*)Kbsr);
    } else {
      auto k = assemble_k_kernel<float>;
      IEDG_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
      hipLaunchKernelGGL(k, dim3(m->nnzb), dim3(STHR), smem, stream, m->b, m->t, m->d_asm_src, (const float*)Ke,
                         (float*)Kbsr);
    }
    IEDG_LAUNCH_CHECK(ctx, "assemble K launch");
  }
  if (R) {
    const int64_t total = m->n_trace;
    hipLaunchKernelGGL(assemble_r_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, m->n_face,
                       m->b, m->t, m->d_face_src, r, G, R);
    IEDG_LAUNCH_CHECK(ctx, "assemble R launch");
  }
  return IEDG_OK;
}

iedg_status iedg_factor_ilu0(iedg_context ctx, iedg_mesh m, iedg_prec prec, const void* Kbsr, void* Mbsr,
                             hipStream_t stream) {
  if (!ctx || !m || !Kbsr || !Mbsr) return IEDG_ERR_INVALID_ARG;
  const size_t es = prec_size(prec);
  if (Kbsr != Mbsr)
    IEDG_HIP(ctx, hipMemcpyAsync(Mbsr, Kbsr, es * m->nnzb * m->b * m->b, hipMemcpyDeviceToDevice, stream));
  const size_t smem = es * m->b * (m->b + 1) + sizeof(int) * 128 + 2 * sizeof(double);
  const size_t tail = sizeof(int) * 128 + 2 * sizeof(double);
  const size_t smem3 = 3 * es * m->b * (m->b + 1) + tail, smem2 = 2 * es * m->b * (m->b + 1) + tail;
  const int mode = smem3 <= 160 * 1024 ? 3 : (smem2 <= 160 * 1024 ? 2 : 0);
  for (int l = 0; l < m->n_levels; ++l) {
    const int r0 = m->level_ptr[l], cnt = m->level_ptr[l + 1] - r0;
    if (mode) {
      const size_t sm = mode == 3 ? smem3 : smem2;
      auto launch = [&](auto kern, auto* Mp) -> iedg_status {
        IEDG_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm));
        hipLaunchKernelGGL(kern, dim3(cnt), dim3(STHR), sm, stream, m->b, m->d_level_rows + r0, m->d_diag_slot,
                           m->d_ilu_lptr, m->d_ilu_l, m->d_ilu_uptr, m->d_ilu_upd, Mp, ctx->d_status);
        return IEDG_OK;
      };
      iedg_status st;
      if (prec == IEDG_F64)
        st = mode == 3 ? launch(ilu0_level_lds_kernel<double, true>, (double*)Mbsr)
                       : launch(ilu0_level_lds_kernel<double, false>, (double*)Mbsr);
      else
        st = mode == 3 ? launch(ilu0_level_lds_kernel<float, true>, (float*)Mbsr)
                       : launch(ilu0_level_lds_kernel<float, false>, (float*)Mbsr);
      if (st != IEDG_OK) return st;
      IEDG_LAUNCH_CHECK(ctx, "ilu0 level launch");
      continue;
    }
    if (prec == IEDG_F64) {
      auto k = ilu0_level_kernel<double>;
      IEDG_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
      hipLaunchKernelGGL(k, dim3(cnt), dim3(STHR), smem, stream, m->b, m->d_level_rows + r0, m->d_diag_slot,
                         m->d_ilu_lptr, m->d_ilu_l, m->d_ilu_uptr, m->d_ilu_upd, (double*)Mbsr, ctx->d_status);
    } else {
      auto k = ilu0_level_kernel<float>;
      IEDG_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
      hipLaunchKernelGGL(k, dim3(cnt), dim3(STHR), smem, stream, m->b, m->d_level_rows + r0, m->d_diag_slot,
                         m->d_ilu_lptr, m->d_ilu_l, m->d_ilu_uptr, m->d_ilu_upd, (float*)Mbsr, ctx->d_status);
    }
    IEDG_LAUNCH_CHECK(ctx, "ilu0 level launch");
  }
  return IEDG_OK;
}

iedg_status iedg_spmv(iedg_context ctx, iedg_mesh m, iedg_prec kprec, const void* K, const double* x, double* y,
                      hipStream_t stream) {
  if (!ctx || !m || !K || !x || !y) return IEDG_ERR_INVALID_ARG;
  return spmv_launch(ctx, m, kprec, K, x, nullptr, y, 0, stream, nullptr);
}

iedg_status iedg_ilu0_apply(iedg_context ctx, iedg_mesh m, iedg_prec mprec, const void* M, const double* x,
                            double* y, hipStream_t stream) {
  if (!ctx || !m || !M || !x || !y) return IEDG_ERR_INVALID_ARG;
  return ilu0_apply_launch(ctx, m, mprec, M, x, y, stream, nullptr);
}

}  // extern "C"
