// Dense b x b block operations shared by the BILU(0) factorisation and the
// MDF ordering: MFMA block products and an in-LDS Gauss-Jordan inverse.
// Blocks are column-major (entry (r, c) at c * b + r), b <= 128, and every
// function is called by all STHR threads of a workgroup.
#pragma once

#include "common.h"

namespace iedg {

constexpr int STHR = 256;

// Product of two b x b column-major blocks with FP64/FP32 MFMA.  Tiles of
// 16 x 16 are dealt to the 4 waves round-robin; each wave keeps up to 8 tile
// accumulators (b <= 128).  mode 0: C = A * B (C may alias A: all products are
// formed before any store, separated by a barrier); mode 1: C -= A * B.
template <typename T>
__device__ void block_mm(int b, const T* A, const T* B, T* C, int mode) {
  typedef Mfma<T> MF;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nt = (b + 15) / 16, ntiles = nt * nt;
  typename MF::acc_t acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = MF::zero();
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int tI = wv + 4 * q;
    if (tI < ntiles) {
      const int i0 = (tI / nt) * 16, j0 = (tI % nt) * 16;
      const int ia = i0 + li, jb = j0 + li;
      for (int k0 = 0; k0 < b; k0 += 4) {
        const int k = k0 + lk;
        const T av = (ia < b && k < b) ? A[(size_t)k * b + ia] : T(0);
        const T bv = (jb < b && k < b) ? B[(size_t)jb * b + k] : T(0);
        acc[q] = MF::mac(av, bv, acc[q]);
      }
    }
  }
  if (mode == 0) __syncthreads();
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int tI = wv + 4 * q;
    if (tI < ntiles) {
      const int i0 = (tI / nt) * 16, j0 = (tI % nt) * 16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + MF::row(lane, v), j = j0 + li;
        if (i < b && j < b) {
          T* c = C + (size_t)j * b + i;
          *c = mode == 0 ? acc[q][v] : *c - acc[q][v];
        }
      }
    }
  }
}

// In-place Gauss-Jordan inverse with partial (row) pivoting of a b x b
// column-major block held in LDS as row-major a[r * (b+1) + c].
template <typename T>
__device__ bool gj_invert(T* a, int b, int* piv, double* rv, int* ri) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int ld = b + 1;
  bool ok = true;
  for (int k = 0; k < b; ++k) {
    if (tid < 64) {
      double best = -1.0;
      int bi = k;
      for (int r = k + lane; r < b; r += 64) {
        const double v = fabs((double)a[r * ld + k]);
        if (v > best) { best = v; bi = r; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(best, off, kWave);
        const int oi = __shfl_xor(bi, off, kWave);
        if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
      }
      if (lane == 0) { rv[0] = best; ri[0] = bi; piv[k] = bi; }
    }
    __syncthreads();
    const int p = ri[0];
    if (!(rv[0] > 0.0) || !isfinite(rv[0])) ok = false;
    if (p != k)
      for (int c = tid; c < b; c += STHR) {
        const T tmp = a[k * ld + c];
        a[k * ld + c] = a[p * ld + c];
        a[p * ld + c] = tmp;
      }
    __syncthreads();
    const T pinv = T(1) / a[k * ld + k];
    __syncthreads();
    if (tid == 0) a[k * ld + k] = T(1);
    __syncthreads();
    for (int c = tid; c < b; c += STHR) a[k * ld + c] *= pinv;
    __syncthreads();
    // eliminate column k from every other row; factors read before update
    for (int q = tid; q < b * b; q += STHR) {
      const int r = q / b, c = q % b;
      if (r != k && c != k) a[r * ld + c] -= a[r * ld + k] * a[k * ld + c];
    }
    __syncthreads();
    for (int r = tid; r < b; r += STHR)
      if (r != k) a[r * ld + k] = -a[r * ld + k] * a[k * ld + k];
    __syncthreads();
  }
  // undo the row interchanges as column interchanges, in reverse order
  for (int k = b - 1; k >= 0; --k) {
    const int p = piv[k];
    if (p != k)
      for (int r = tid; r < b; r += STHR) {
        const T tmp = a[r * ld + k];
        a[r * ld + k] = a[r * ld + p];
        a[r * ld + p] = tmp;
      }
    __syncthreads();
  }
  return ok;
}


}  // namespace iedg
