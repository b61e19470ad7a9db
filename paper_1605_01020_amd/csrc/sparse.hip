// Block-sparse trace system on gfx950: assembly of K and R (section 2.2.1,
// eq. LS), BILU(0) factorisation and its triangular sweeps, and the BSR
// matrix-vector product (section 2.2.2).  Blocks are b x b, column-major,
// stored in the row order of the mesh's ordering (see iedg.h).
#include <cfloat>

#include "blockops.h"
#include "common.h"
#include "mesh.h"

namespace iedg {

// ---- assembly ----------------------------------------------------------
// Block s of K is the sum, in list order (ascending element, then local
// slots), of the sub-blocks Ke_e[a*b:(a+1)*b, c*b:(c+1)*b] (row-major t x t)
// coded e*S*S + a*S + c in asm_list[asm_ptr[s] .. asm_ptr[s+1]).
__device__ __forceinline__ size_t asm_offset(int code, int S, int b, int t) {
  const int e = code / (S * S), ac = code - e * S * S, a = ac / S, c = ac - a * S;
  return (size_t)e * t * t + (size_t)a * b * t + (size_t)c * b;
}

// One workgroup per block (face units): the summed block is transposed to
// column-major through LDS.
template <typename T>
__global__ __launch_bounds__(STHR) void assemble_k_kernel(int b, int t, int S, const int32_t* asm_ptr,
                                                          const int32_t* asm_list, const T* Ke, T* Kbsr) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* tile = reinterpret_cast<T*>(smem_raw);  // b x (b+1)
  const int64_t s = blockIdx.x;
  const int k0 = asm_ptr[s], k1 = asm_ptr[s + 1];
  const int bb = b * b;
  for (int i0 = threadIdx.x; i0 < bb; i0 += STHR * 8) {
    T v[8];
    for (int k = k0; k < k1; ++k) {
      const T* p = Ke + asm_offset(asm_list[k], S, b, t);
      T x[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int i = i0 + STHR * j;
        x[j] = i < bb ? p[(size_t)(i / b) * t + i % b] : T(0);
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = k == k0 ? x[j] : v[j] + x[j];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = i0 + STHR * j;
      if (i < bb) tile[(i / b) * (b + 1) + i % b] = v[j];
    }
  }
  __syncthreads();
  T* out = Kbsr + (size_t)s * bb;
  for (int i = threadIdx.x; i < bb; i += STHR) {
    const int cc = i / b, rr = i % b;
    out[i] = tile[rr * (b + 1) + cc];
  }
}

// Small blocks (node units): one thread per block entry, written directly
// in column-major order; same summation order.
template <typename T>
__global__ void assemble_k_small_kernel(int b, int t, int S, int64_t nnzb, const int32_t* asm_ptr,
                                        const int32_t* asm_list, const T* Ke, T* Kbsr) {
  const int bb = b * b;
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= nnzb * bb) return;
  const int64_t s = x / bb;
  const int i = (int)(x - s * bb), cc = i / b, rr = i - cc * b;
  T v = T(0);
  for (int k = asm_ptr[s]; k < asm_ptr[s + 1]; ++k) {
    const T y = Ke[asm_offset(asm_list[k], S, b, t) + (size_t)rr * t + cc];
    v = k == asm_ptr[s] ? y : v + y;
  }
  Kbsr[x] = v;
}

// R[u*b + l] = G[u*b + l] + sum, in list order (ascending e, a), of
// r_e[a*b + l] over the slots coded e*S + a in src_list[src_ptr[u] ..].
__global__ void assemble_r_kernel(int n_face, int b, int t, int S, const int32_t* src_ptr, const int32_t* src_list,
                                  const double* r, const double* G, double* R) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n_face * b) return;
  const int f = (int)(i / b), l = (int)(i % b);
  double v = G ? G[i] : 0.0;
  if (r) {
    for (int k = src_ptr[f]; k < src_ptr[f + 1]; ++k) {
      const int code = src_list[k], e = code / S, a = code - e * S;
      v += r[(size_t)e * t + a * b + l];
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

// One level of the BILU(0) sweeps (rows[n_copy ..] of the launch):
//   mode 0, forward:           y_i = x_i - sum over lower slots L_ik v_k;
//   mode 1, backward:          y_i = Uinv_i (y_i - sum over upper slots U_ij v_j);
//   mode 2, forward + inverse: y_i = Uinv_i (x_i - sum over lower slots L_ik v_k),
//           for the last level, whose rows have no upper slots;
// v is y, or x where every summed neighbour lies in level 0 (whose forward
// values equal x).  The first n_copy workgroups copy y_i = x_i for the rows
// of level 0, which have no lower slots, so that level 0 and level 1 share a
// launch.  x may equal y.
template <typename T>
__global__ __launch_bounds__(STHR) void sweep_kernel(int b, const int32_t* rows, const int32_t* row_face,
                                                     const int32_t* row_ptr, const int32_t* diag_slot,
                                                     const int32_t* col_face, const T* M, const double* x,
                                                     double* y, const double* v, int mode, int n_copy,
                                                     const int* skip) {
  __shared__ double red[STHR + 128];
  if (skip && *skip) return;
  const int i = rows[blockIdx.x];
  const size_t o = (size_t)row_face[i] * b;
  if ((int)blockIdx.x < n_copy) {
    if (x != y && threadIdx.x < b) y[o + threadIdx.x] = x[o + threadIdx.x];
    return;
  }
  const int G = STHR / b, g = threadIdx.x / b, rr = threadIdx.x % b;
  const int ds = diag_slot[i];
  const int s0 = mode == 1 ? ds + 1 : row_ptr[i];
  const int s1 = mode == 1 ? row_ptr[i + 1] : ds;
  const double* base = mode == 1 ? y : x;
  const double sum = block_row_sum<T>(b, M, col_face, s0, s1, v, g, G, rr);
  group_reduce(red, b, G, g, rr, sum);
  if (mode == 0) {
    if (threadIdx.x < b) y[o + threadIdx.x] = base[o + threadIdx.x] - red[G * b + threadIdx.x];
    return;
  }
  // s = base_i - sum  ->  svec; then y_i = Uinv s
  __shared__ double svec[128];
  if (threadIdx.x < b) svec[threadIdx.x] = base[o + threadIdx.x] - red[G * b + threadIdx.x];
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
// One workgroup of FTHR threads per block row i of a level (section 2.2.2,
// BILU(0)).  For each lower slot (i, k) in elimination order:
//   L_ik = A_ik U_kk^{-1}          (A_ik staged row-major in LDS, the product
//                                   written to LDS and to M),
//   A_ij -= L_ik U_kj              (every j of the row coupled to k),
// then the pivot block A_ii is inverted in place.  Block products are split
// into strips of 16 columns: a wave forms one strip (all b rows) with 16x16x4
// MFMA, its A fragments read from LDS as 4-vectors and its B fragments (4
// consecutive k of one column of a column-major block) loaded from HBM as
// vectors; the k index of the four MFMAs of a vector is permuted between
// lanes, which reorders only the sum.  Strips of all updates of one slot are
// dealt to the 8 waves.  The inversion is Gauss-Jordan with partial pivoting
// in exchange form, the block held in registers (4 threads per row, CPT
// columns each) with one workgroup barrier per column: each wave posts its
// best candidate row to LDS, so after the barrier every thread knows the
// pivot row without a second exchange.
constexpr int FTHR = 512;

template <typename T, int NB>
struct FactorSmem {
  static constexpr int lda = 16 * NB + 4;   // row stride of the row-major block (16-byte rows)
  static constexpr int slot = 16 * NB;      // one posted candidate row
  static constexpr size_t y_bytes = sizeof(T) * (size_t)(16 * NB) * lda;
  static constexpr size_t slot_bytes = sizeof(T) * 2 * 8 * slot;
  static constexpr size_t bytes = y_bytes + slot_bytes + 2 * 8 * sizeof(uint32_t) + 128 * sizeof(int);
};

template <typename T> struct Vec4;
template <> struct Vec4<float> { typedef f4 type; };
template <> struct Vec4<double> { typedef d4 type; };

// Row of the A fragment supplied by lane li so that the accumulator lane
// (li, lg) holds rows 4 lg .. 4 lg + 3 of its column (FP64 MFMA lays its
// output rows out as lg + 4 v).
template <typename T>
__device__ __forceinline__ int frag_row(int li) {
  return sizeof(T) == 8 ? 4 * (li & 3) + (li >> 2) : li;
}

// Y[r * lda + c] = G[c * b + r] for r, c < b (a column-major block to
// row-major LDS), 4 loads in flight per thread.
template <typename T, int NB>
__device__ __forceinline__ void stage_rowmajor(const T* __restrict__ G, T* Y, int b) {
  constexpr int lda = FactorSmem<T, NB>::lda;
  const int bb = b * b;
  for (int q0 = threadIdx.x; q0 < bb; q0 += FTHR * 4) {
    T v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = q0 + FTHR * j;
      v[j] = q < bb ? G[q] : T(0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = q0 + FTHR * j;
      if (q < bb) {
        const int c = q / b, r = q - c * b;
        Y[r * lda + c] = v[j];
      }
    }
  }
}

// B fragment of chunk c: B[16 c + 4 lg + s][j], s = 0..3 (zero past b).
template <typename T, bool VEC>
__device__ __forceinline__ typename Vec4<T>::type load_bfrag(const T* __restrict__ B, int b, int j, int k0) {
  typedef typename Vec4<T>::type V4;
  V4 x = V4{T(0), T(0), T(0), T(0)};
  if constexpr (VEC) {
    if (j < b && k0 < b) x = *reinterpret_cast<const V4*>(B + (size_t)j * b + k0);
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s)
      if (j < b && k0 + s < b) x[s] = B[(size_t)j * b + k0 + s];
  }
  return x;
}

// acc[q] = (Y B)[16 q .. 16 q + 15, j0 .. j0 + 15] for q < NB: Y row-major in
// LDS (rows and columns past b zero), B a column-major b x b block in HBM.
// The next chunk's B fragment is loaded while the current one is consumed;
// tile rows are taken in pairs so that consecutive MFMAs are independent.
template <typename T, int NB, bool VEC>
__device__ __forceinline__ void strip_mm(const T* Y, const T* __restrict__ B, int b, int j0,
                                         typename Mfma<T>::acc_t (&acc)[NB]) {
  typedef Mfma<T> MF;
  typedef typename Vec4<T>::type V4;
  constexpr int lda = FactorSmem<T, NB>::lda;
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  const int j = j0 + li;
#pragma unroll
  for (int q = 0; q < NB; ++q) acc[q] = MF::zero();
  const T* yrow = Y + frag_row<T>(li) * lda + 4 * lg;
  V4 bn = load_bfrag<T, VEC>(B, b, j, 4 * lg);
  // a rolled chunk loop keeps one chunk's A fragments live (unrolled, the
  // scheduler hoists every chunk's LDS reads and runs out of registers)
#pragma unroll 1
  for (int c = 0; c < NB; ++c) {
    const V4 bc = bn;
    if (c + 1 < NB) bn = load_bfrag<T, VEC>(B, b, j, 16 * (c + 1) + 4 * lg);
#pragma unroll
    for (int q = 0; q < NB; q += 2) {
      const V4 a0 = *reinterpret_cast<const V4*>(yrow + 16 * q * lda + 16 * c);
      if (q + 1 < NB) {
        const V4 a1 = *reinterpret_cast<const V4*>(yrow + 16 * (q + 1) * lda + 16 * c);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          acc[q] = MF::mac(a0[s], bc[s], acc[q]);
          acc[q + 1] = MF::mac(a1[s], bc[s], acc[q + 1]);
        }
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) acc[q] = MF::mac(a0[s], bc[s], acc[q]);
      }
    }
  }
}

// C = acc (sub false) or C -= acc (sub true) on the accumulator rows
// 16 q + 4 lg .. + 3 of column j0 + li (rows and columns past b skipped).
template <typename T, int NB, bool VEC>
__device__ __forceinline__ void strip_rmw(T* C, int b, int j0, const typename Mfma<T>::acc_t (&acc)[NB], bool sub) {
  typedef typename Vec4<T>::type V4;
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  const int j = j0 + li;
  if (j >= b) return;
  T* col = C + (size_t)j * b;
  if constexpr (VEC) {
    V4 x[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int i0 = 16 * q + 4 * lg;
      if (sub && i0 < b) x[q] = *reinterpret_cast<const V4*>(col + i0);
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int i0 = 16 * q + 4 * lg;
      if (i0 < b) {
        V4 y;
#pragma unroll
        for (int v = 0; v < 4; ++v) y[v] = sub ? x[q][v] - acc[q][v] : acc[q][v];
        *reinterpret_cast<V4*>(col + i0) = y;
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * q + 4 * lg + v;
        if (i < b) col[i] = sub ? col[i] - acc[q][v] : acc[q][v];
      }
  }
}

template <typename T, int NB, bool VEC>
__global__ __launch_bounds__(FTHR) void ilu0_row_kernel(int b, const int32_t* __restrict__ rows,
                                                        const int32_t* __restrict__ diag_slot,
                                                        const int32_t* __restrict__ lptr,
                                                        const int32_t* __restrict__ lslot,
                                                        const int32_t* __restrict__ uptr,
                                                        const int32_t* __restrict__ upd, T* M,
                                                        DeviceStatus* status) {
  typedef Mfma<T> MF;
  typedef FactorSmem<T, NB> SM;
  typedef typename Vec4<T>::type V4;
  constexpr int lda = SM::lda, CPT = 4 * NB;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Y = reinterpret_cast<T*>(smem_raw);
  T* slots = reinterpret_cast<T*>(smem_raw + SM::y_bytes);                   // [2][8][16 NB]
  uint32_t* skey = reinterpret_cast<uint32_t*>(smem_raw + SM::y_bytes + SM::slot_bytes);  // [2][8]
  int* prow = reinterpret_cast<int*>(skey + 16);                                         // [128]
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int i = rows[blockIdx.x];
  const size_t bb = (size_t)b * b;
  // rows and columns of Y past b stay zero (finite operands where k >= b)
  for (int q = tid; q < 16 * NB * lda; q += FTHR) Y[q] = T(0);
  __syncthreads();
  typename MF::acc_t acc[NB];
  for (int l = lptr[i]; l < lptr[i + 1]; ++l) {
    const int sik = lslot[2 * l], dk = lslot[2 * l + 1];
    T* Aik = M + (size_t)sik * bb;
    stage_rowmajor<T, NB>(Aik, Y, b);
    __syncthreads();
    if (wv < NB) strip_mm<T, NB, VEC>(Y, M + (size_t)dk * bb, b, 16 * wv, acc);
    __syncthreads();  // every wave has read A_ik from Y
    if (wv < NB) {
      strip_rmw<T, NB, VEC>(Aik, b, 16 * wv, acc, false);
      const int li = lane & 15, lg = lane >> 4, j = 16 * wv + li;
      if (j < b)
#pragma unroll
        for (int q = 0; q < NB; ++q)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = 16 * q + 4 * lg + v;
            if (r < b) Y[r * lda + j] = acc[q][v];
          }
    }
    __syncthreads();  // L_ik in Y
    const int u0 = uptr[l], nu = uptr[l + 1] - u0;
    for (int w = wv; w < nu * NB; w += FTHR / 64) {
      const int u = u0 + w / NB, c = w - (w / NB) * NB;
      strip_mm<T, NB, VEC>(Y, M + (size_t)upd[2 * u] * bb, b, 16 * c, acc);
      strip_rmw<T, NB, VEC>(M + (size_t)upd[2 * u + 1] * bb, b, 16 * c, acc, true);
    }
    sync_global();  // the next slot reads blocks other waves updated
  }
  // ---- pivot block: Gauss-Jordan inverse in exchange form ----
  T* Dg = M + (size_t)diag_slot[i] * bb;
  stage_rowmajor<T, NB>(Dg, Y, b);
  __syncthreads();
  const int r = tid >> 2, h = tid & 3;  // row r, columns h CPT .. h CPT + CPT - 1
  const bool live = r < b;
  T W[CPT];
#pragma unroll
  for (int j = 0; j < CPT; j += 4) {
    V4 x = V4{T(0), T(0), T(0), T(0)};
    if (r < 16 * NB) x = *reinterpret_cast<const V4*>(Y + r * lda + h * CPT + j);
#pragma unroll
    for (int s = 0; s < 4; ++s) W[j + s] = x[s];
  }
  bool pivoted = false, ok = true;
  int mystep = -1;
  // Waves past the last row (b <= 16 NB rows, 16 rows a wave) only keep the
  // barriers.  A candidate's key is its magnitude in FP32 with the low 8
  // mantissa bits replaced by 255 - row (never zero, which marks "no
  // candidate"): the largest key is the largest magnitude to 2^-15
  // relative, ties to the smaller row (the pivot must only
  // be near the column maximum for stability, and equal keys give the same
  // choice on every run).  NaN and Inf are taken first, and flagged.
  const bool active = wv < NB;
  for (int hk = 0; hk < 4; ++hk) {
#pragma unroll
    for (int kk = 0; kk < CPT; ++kk) {
      const int k = hk * CPT + kk;
      if (k < b) {
        const int par = k & 1;
        T v = T(0);
        if (active) {
          v = __shfl(W[kk], (lane & ~3) | hk, kWave);  // entry (r, k)
          float fm = fabsf((float)v);
          if (!(fm <= FLT_MAX)) fm = INFINITY;
          uint32_t key = (live && !pivoted) ? ((__float_as_uint(fm) & ~255u) | (uint32_t)(255 - r)) : 0u;
#pragma unroll
          for (int off = 4; off < 64; off <<= 1) key = max(key, (uint32_t)__shfl_xor((int)key, off, kWave));
          if (key != 0u && r == 255 - (int)(key & 255u)) {
            T* sl = slots + (par * 8 + wv) * SM::slot + h * CPT;
#pragma unroll
            for (int j = 0; j < CPT; j += 4) *reinterpret_cast<V4*>(sl + j) = V4{W[j], W[j + 1], W[j + 2], W[j + 3]};
          }
          if (lane == 0) skey[par * 8 + wv] = key;
        }
        __syncthreads();
        if (active) {
          uint32_t best = skey[par * 8];
#pragma unroll
          for (int w = 1; w < NB; ++w) best = max(best, skey[par * 8 + w]);
          const int p = 255 - (int)(best & 255u);
          const T* ps = slots + (par * 8 + (p >> 4)) * SM::slot;
          const T piv = ps[k];
          if (!(piv != T(0)) || !(fabs((double)piv) <= DBL_MAX)) ok = false;
          const T ip = T(1) / piv;
          const T c = -(v * ip);
          // every row: W(r, c') -= W(r, k) W(p, c') / W(p, k)
#pragma unroll
          for (int j = 0; j < CPT; j += 4) {
            const V4 x = *reinterpret_cast<const V4*>(ps + h * CPT + j);
#pragma unroll
            for (int s = 0; s < 4; ++s) W[j + s] = fma(c, x[s], W[j + s]);
          }
          const bool me = r == p;
          if (me) {  // the pivot row: W(p, c') = -W(p, c') / W(p, k)
#pragma unroll
            for (int j = 0; j < CPT; j += 4) {
              const V4 x = *reinterpret_cast<const V4*>(ps + h * CPT + j);
#pragma unroll
              for (int s = 0; s < 4; ++s) W[j + s] = -(x[s] * ip);
            }
            pivoted = true;
            mystep = k;
          }
          if (h == hk) W[kk] = me ? ip : v * ip;  // column k: 1 / W(p, k) and W(r, k) / W(p, k)
          if (tid == 0) prow[k] = p;
        }
      }
    }
  }
  __syncthreads();  // prow complete; Y no longer read
  // inverse(step(r), prow[c]) = W(r, c), staged column-major in Y
  if (live && mystep >= 0)
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      const int c = h * CPT + j;
      if (c < b) Y[prow[c] * b + mystep] = W[j];
    }
  __syncthreads();
  for (int q = tid; q < (int)bb; q += FTHR) Dg[q] = Y[q];
  if (!ok && tid == 0) latch_status(status, IEDG_ERR_SINGULAR, i);
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
// With sweep_fused (the last level has no upper slots) level 0's forward
// step, a copy, shares a launch with level 1, and the last level's forward
// and backward steps run as one: 2 L - 2 launches for L >= 2 levels instead
// of 2 L, with bitwise the same result (level 0's forward values are x
// exactly, and the last level's backward sum is empty).
template <typename T>
static void sweep_launch(iedg_mesh m, int l0, int l1, int n_copy, const T* M, const double* x, double* y,
                         const double* v, int mode, hipStream_t stream, const int* skip) {
  const int r0 = m->level_ptr[l0], cnt = m->level_ptr[l1] - r0;
  hipLaunchKernelGGL(sweep_kernel<T>, dim3(cnt), dim3(STHR), 0, stream, m->b, m->d_level_rows + r0,
                     m->d_row_face, m->d_row_ptr, m->d_diag_slot, m->d_col_face, M, x, y, v, mode, n_copy, skip);
}

template <typename T>
static void ilu0_apply_levels(iedg_mesh m, const T* M, const double* x, double* y, hipStream_t stream,
                              const int* skip) {
  const int L = m->n_levels;
  if (L == 0) return;
  if (!m->sweep_fused) {
    for (int l = 0; l < L; ++l) sweep_launch<T>(m, l, l + 1, 0, M, x, y, y, 0, stream, skip);
    for (int l = L - 1; l >= 0; --l) sweep_launch<T>(m, l, l + 1, 0, M, y, y, y, 1, stream, skip);
    return;
  }
  if (L == 1) {
    sweep_launch<T>(m, 0, 1, 0, M, x, y, y, 2, stream, skip);
    return;
  }
  // levels 0 and 1: level 1 sums over level-0 neighbours only, read from x
  const int cnt0 = m->level_ptr[1] - m->level_ptr[0];
  sweep_launch<T>(m, 0, 2, cnt0, M, x, y, x, L == 2 ? 2 : 0, stream, skip);
  for (int l = 2; l < L; ++l) sweep_launch<T>(m, l, l + 1, 0, M, x, y, y, l == L - 1 ? 2 : 0, stream, skip);
  for (int l = L - 2; l >= 0; --l) sweep_launch<T>(m, l, l + 1, 0, M, y, y, y, 1, stream, skip);
}

iedg_status ilu0_apply_launch(iedg_context ctx, iedg_mesh m, iedg_prec mprec, const void* M, const double* x,
                              double* y, hipStream_t stream, const int* skip) {
  if (mprec == IEDG_F64)
    ilu0_apply_levels<double>(m, (const double*)M, x, y, stream, skip);
  else
    ilu0_apply_levels<float>(m, (const float*)M, x, y, stream, skip);
  IEDG_LAUNCH_CHECK(ctx, "ilu0 sweep launch");
  return IEDG_OK;
}

}  // namespace iedg

// ---- BILU(0) of small blocks (b <= 8: the m x m node blocks of the IEDG
// numbering) ----------------------------------------------------------------
// One wave per block row (4 rows a workgroup, no barriers).  For each lower
// slot (i, k) in elimination order every lane forms L_ik = A_ik U_kk^{-1} in
// registers (the blocks are broadcast loads); lane 0 stores it, and the
// updates A_ij -= L_ik U_kj of that slot are dealt to the lanes, one block
// each.  The updated blocks are made visible to the whole wave (stores
// complete, vector L1 invalidated) before the next slot reads its A_ik.
// Lane 0 then inverts the pivot block by Gauss-Jordan with partial pivoting
// in exchange form (no row moves: the inverse is written through the
// recorded pivot rows and steps).
template <typename T, int B>
__device__ __forceinline__ void small_load(const T* __restrict__ p, T (&x)[B * B]) {
#pragma unroll
  for (int q = 0; q < B * B; ++q) x[q] = p[q];
}

// C = A B (column-major b x b: entry (r, c) at c B + r), or C -= A B.
template <typename T, int B, bool SUB>
__device__ __forceinline__ void small_mm(const T (&a)[B * B], const T (&b)[B * B], T (&c)[B * B]) {
#pragma unroll
  for (int col = 0; col < B; ++col)
#pragma unroll
    for (int r = 0; r < B; ++r) {
      T v = T(0);
#pragma unroll
      for (int k = 0; k < B; ++k) v += a[k * B + r] * b[col * B + k];
      c[col * B + r] = SUB ? c[col * B + r] - v : v;
    }
}

template <typename T, int B>
__global__ __launch_bounds__(256) void ilu0_small_kernel(int nrows, const int32_t* __restrict__ rows,
                                                         const int32_t* __restrict__ diag_slot,
                                                         const int32_t* __restrict__ lptr,
                                                         const int32_t* __restrict__ lslot,
                                                         const int32_t* __restrict__ uptr,
                                                         const int32_t* __restrict__ upd, T* M,
                                                         DeviceStatus* status) {
  constexpr int BB = B * B;
  const int lane = threadIdx.x & 63;
  const int rr = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (rr >= nrows) return;
  const int i = rows[rr];
  const int l0 = lptr[i], l1 = lptr[i + 1];
  // read-only operands of the next slot (its U_kk^{-1} and this lane's first
  // U_kj, from rows of earlier levels) are loaded one slot ahead; A_ik and
  // the lane's first A_ij are loaded together right after the previous
  // slot's updates are visible
  T un[BB], ukn[BB];
  if (l0 < l1) {
    small_load<T, B>(M + (size_t)lslot[2 * l0 + 1] * BB, un);
    const int x0 = uptr[l0] + lane;
    if (x0 < uptr[l0 + 1]) small_load<T, B>(M + (size_t)upd[2 * x0] * BB, ukn);
  }
  for (int l = l0; l < l1; ++l) {
    const int sik = lslot[2 * l];
    const int xb = uptr[l], xe = uptr[l + 1];
    T a[BB], u[BB], L[BB], uk0[BB], c0[BB];
    small_load<T, B>(M + (size_t)sik * BB, a);
    if (xb + lane < xe) small_load<T, B>(M + (size_t)upd[2 * (xb + lane) + 1] * BB, c0);
#pragma unroll
    for (int q = 0; q < BB; ++q) {
      u[q] = un[q];
      uk0[q] = ukn[q];
    }
    if (l + 1 < l1) {
      small_load<T, B>(M + (size_t)lslot[2 * (l + 1) + 1] * BB, un);
      const int x1 = xe + lane;
      if (x1 < uptr[l + 2]) small_load<T, B>(M + (size_t)upd[2 * x1] * BB, ukn);
    }
    small_mm<T, B, false>(a, u, L);
    if (lane == 0)
#pragma unroll
      for (int q = 0; q < BB; ++q) M[(size_t)sik * BB + q] = L[q];
    if (xb + lane < xe) {
      small_mm<T, B, true>(L, uk0, c0);
      T* C = M + (size_t)upd[2 * (xb + lane) + 1] * BB;
#pragma unroll
      for (int q = 0; q < BB; ++q) C[q] = c0[q];
    }
    for (int x = xb + lane + 64; x < xe; x += 64) {
      T* C = M + (size_t)upd[2 * x + 1] * BB;
      T ukj[BB], c[BB];
      small_load<T, B>(M + (size_t)upd[2 * x] * BB, ukj);
      small_load<T, B>(C, c);
      small_mm<T, B, true>(L, ukj, c);
#pragma unroll
      for (int q = 0; q < BB; ++q) C[q] = c[q];
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    asm volatile("buffer_inv sc0" ::: "memory");
  }
  if (lane != 0) return;
  T* Dg = M + (size_t)diag_slot[i] * BB;
  T W[B][B];
#pragma unroll
  for (int r = 0; r < B; ++r)
#pragma unroll
    for (int c = 0; c < B; ++c) W[r][c] = Dg[c * B + r];
  bool piv[B];
  int step[B], prow[B];
#pragma unroll
  for (int r = 0; r < B; ++r) {
    piv[r] = false;
    step[r] = 0;
  }
  bool ok = true;
#pragma unroll
  for (int k = 0; k < B; ++k) {
    // largest magnitude in column k among unpivoted rows, ties to the smaller
    // row; NaN is never larger, so the first unpivoted row stands in
    int p = -1;
    double best = -1.0;
#pragma unroll
    for (int r = 0; r < B; ++r) {
      const double v = fabs((double)W[r][k]);
      if (!piv[r] && (p < 0 || v > best)) {
        best = v;
        p = r;
      }
    }
    if (!(best > 0.0) || !(best <= DBL_MAX)) ok = false;
    T pr[B];
#pragma unroll
    for (int c = 0; c < B; ++c) {
      T v = W[0][c];
#pragma unroll
      for (int r = 1; r < B; ++r) v = r == p ? W[r][c] : v;
      pr[c] = v;
    }
    const T ip = T(1) / pr[k];
#pragma unroll
    for (int r = 0; r < B; ++r) {
      if (r == p) {
#pragma unroll
        for (int c = 0; c < B; ++c) W[r][c] = c == k ? ip : -(pr[c] * ip);
        piv[r] = true;
        step[r] = k;
      } else {
        const T v = W[r][k];
#pragma unroll
        for (int c = 0; c < B; ++c) W[r][c] = c == k ? v * ip : W[r][c] - v * (pr[c] * ip);
      }
    }
    prow[k] = p;
  }
  // inverse(step(r), prow(c)) = W(r, c)
#pragma unroll
  for (int r = 0; r < B; ++r)
#pragma unroll
    for (int c = 0; c < B; ++c) Dg[prow[c] * B + step[r]] = W[r][c];
  if (!ok) latch_status(status, IEDG_ERR_SINGULAR, i);
}

// The same factorisation with the row's blocks staged in LDS: one wave per
// block row (one row a workgroup).  Every slot of row i (A_ik, the updated
// A_ij, the pivot block) lives in LDS from the first read to the final
// write-back, so the chain of lower slots runs without the global stores,
// waits and cache invalidations between slots; only U_kk^{-1} and U_kj
// (rows of earlier levels) come from global memory, one slot ahead as in
// ilu0_small_kernel.  The arithmetic is that kernel's, operation for
// operation.  Dynamic LDS: the longest row of the level, in blocks.
template <typename T, int B>
__global__ __launch_bounds__(64) void ilu0_small_lds_kernel(const int32_t* __restrict__ rows,
                                                            const int32_t* __restrict__ row_ptr,
                                                            const int32_t* __restrict__ diag_slot,
                                                            const int32_t* __restrict__ lptr,
                                                            const int32_t* __restrict__ lslot,
                                                            const int32_t* __restrict__ uptr,
                                                            const int32_t* __restrict__ upd, T* M,
                                                            DeviceStatus* status) {
  constexpr int BB = B * B;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* R = reinterpret_cast<T*>(lds_raw);
  const int lane = threadIdx.x;
  const int i = rows[blockIdx.x];
  const int s0 = row_ptr[i], nv = (row_ptr[i + 1] - s0) * BB;
  const T* Mrow = M + (size_t)s0 * BB;
  for (int q = lane; q < nv; q += 64) R[q] = Mrow[q];
  const int l0 = lptr[i], l1 = lptr[i + 1];
  T un[BB], ukn[BB];
  if (l0 < l1) {
    small_load<T, B>(M + (size_t)lslot[2 * l0 + 1] * BB, un);
    const int x0 = uptr[l0] + lane;
    if (x0 < uptr[l0 + 1]) small_load<T, B>(M + (size_t)upd[2 * x0] * BB, ukn);
  }
  __syncthreads();
  for (int l = l0; l < l1; ++l) {
    const int sik = lslot[2 * l] - s0;
    const int xb = uptr[l], xe = uptr[l + 1];
    T a[BB], u[BB], L[BB], uk0[BB], c0[BB];
    small_load<T, B>(R + sik * BB, a);
    if (xb + lane < xe) small_load<T, B>(R + (upd[2 * (xb + lane) + 1] - s0) * BB, c0);
#pragma unroll
    for (int q = 0; q < BB; ++q) {
      u[q] = un[q];
      uk0[q] = ukn[q];
    }
    if (l + 1 < l1) {
      small_load<T, B>(M + (size_t)lslot[2 * (l + 1) + 1] * BB, un);
      const int x1 = xe + lane;
      if (x1 < uptr[l + 2]) small_load<T, B>(M + (size_t)upd[2 * x1] * BB, ukn);
    }
    small_mm<T, B, false>(a, u, L);
    if (xb + lane < xe) {
      small_mm<T, B, true>(L, uk0, c0);
      T* C = R + (upd[2 * (xb + lane) + 1] - s0) * BB;
#pragma unroll
      for (int q = 0; q < BB; ++q) C[q] = c0[q];
    }
    for (int x = xb + lane + 64; x < xe; x += 64) {
      T* C = R + (upd[2 * x + 1] - s0) * BB;
      T ukj[BB], c[BB];
      small_load<T, B>(M + (size_t)upd[2 * x] * BB, ukj);
      small_load<T, B>(C, c);
      small_mm<T, B, true>(L, ukj, c);
#pragma unroll
      for (int q = 0; q < BB; ++q) C[q] = c[q];
    }
    // every lane has read A_ik (into a) before lane 0 replaces it by L_ik;
    // the updates of this slot are visible before the next slot reads
    __syncthreads();
    if (lane == 0)
#pragma unroll
      for (int q = 0; q < BB; ++q) R[sik * BB + q] = L[q];
    __syncthreads();
  }
  if (lane == 0) {
    T* Dg = R + (diag_slot[i] - s0) * BB;
    T W[B][B];
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
      for (int c = 0; c < B; ++c) W[r][c] = Dg[c * B + r];
    bool piv[B];
    int step[B], prow[B];
#pragma unroll
    for (int r = 0; r < B; ++r) {
      piv[r] = false;
      step[r] = 0;
    }
    bool ok = true;
#pragma unroll
    for (int k = 0; k < B; ++k) {
      int p = -1;
      double best = -1.0;
#pragma unroll
      for (int r = 0; r < B; ++r) {
        const double v = fabs((double)W[r][k]);
        if (!piv[r] && (p < 0 || v > best)) {
          best = v;
          p = r;
        }
      }
      if (!(best > 0.0) || !(best <= DBL_MAX)) ok = false;
      T pr[B];
#pragma unroll
      for (int c = 0; c < B; ++c) {
        T v = W[0][c];
#pragma unroll
        for (int r = 1; r < B; ++r) v = r == p ? W[r][c] : v;
        pr[c] = v;
      }
      const T ip = T(1) / pr[k];
#pragma unroll
      for (int r = 0; r < B; ++r) {
        if (r == p) {
#pragma unroll
          for (int c = 0; c < B; ++c) W[r][c] = c == k ? ip : -(pr[c] * ip);
          piv[r] = true;
          step[r] = k;
        } else {
          const T v = W[r][k];
#pragma unroll
          for (int c = 0; c < B; ++c) W[r][c] = c == k ? v * ip : W[r][c] - v * (pr[c] * ip);
        }
      }
      prow[k] = p;
    }
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
      for (int c = 0; c < B; ++c) Dg[prow[c] * B + step[r]] = W[r][c];
    if (!ok) latch_status(status, IEDG_ERR_SINGULAR, i);
  }
  __syncthreads();
  T* Mw = M + (size_t)s0 * BB;
  for (int q = lane; q < nv; q += 64) Mw[q] = R[q];
}

// LDS a workgroup of ilu0_small_lds_kernel may take (the rest of the CU's
// 160 KiB stays for other rows of the level).
constexpr size_t kSmallRowLds = 96 * 1024;

template <typename T, int B>
static iedg_status factor_levels_small(iedg_context ctx, iedg_mesh m, T* M, hipStream_t stream) {
  auto kern = ilu0_small_kernel<T, B>;
  auto kern_lds = ilu0_small_lds_kernel<T, B>;
  const size_t blk = sizeof(T) * B * B;
  IEDG_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void*>(kern_lds),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmallRowLds));
  for (int l = 0; l < m->n_levels; ++l) {
    const int r0 = m->level_ptr[l], cnt = m->level_ptr[l + 1] - r0;
    if (cnt == 0) continue;
    // the longest row of the level decides the LDS of every workgroup
    int len = 0;
    for (int r = r0; r < r0 + cnt; ++r) {
      const int i = m->level_rows[r];
      len = std::max(len, m->row_ptr[i + 1] - m->row_ptr[i]);
    }
    const size_t lds = blk * (size_t)len;
    if (lds <= kSmallRowLds) {
      hipLaunchKernelGGL(kern_lds, dim3(cnt), dim3(64), lds, stream, m->d_level_rows + r0, m->d_row_ptr,
                         m->d_diag_slot, m->d_ilu_lptr, m->d_ilu_l, m->d_ilu_uptr, m->d_ilu_upd, M, ctx->d_status);
    } else {
      hipLaunchKernelGGL(kern, dim3((cnt + 3) / 4), dim3(256), 0, stream, cnt,
                         m->d_level_rows + r0, m->d_diag_slot, m->d_ilu_lptr, m->d_ilu_l, m->d_ilu_uptr,
                         m->d_ilu_upd, M, ctx->d_status);
    }
    IEDG_LAUNCH_CHECK(ctx, "ilu0 small level launch");
  }
  return IEDG_OK;
}

template <typename T, int NB>
static iedg_status factor_levels_nb(iedg_context ctx, iedg_mesh m, T* M, hipStream_t stream) {
  const size_t smem = FactorSmem<T, NB>::bytes;
  auto kern = (m->b % 4 == 0) ? ilu0_row_kernel<T, NB, true> : ilu0_row_kernel<T, NB, false>;
  IEDG_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)smem));
  for (int l = 0; l < m->n_levels; ++l) {
    const int r0 = m->level_ptr[l], cnt = m->level_ptr[l + 1] - r0;
    if (cnt == 0) continue;
    hipLaunchKernelGGL(kern, dim3(cnt), dim3(FTHR), smem, stream, m->b, m->d_level_rows + r0, m->d_diag_slot,
                       m->d_ilu_lptr, m->d_ilu_l, m->d_ilu_uptr, m->d_ilu_upd, M, ctx->d_status);
    IEDG_LAUNCH_CHECK(ctx, "ilu0 level launch");
  }
  return IEDG_OK;
}

template <typename T>
static iedg_status factor_levels(iedg_context ctx, iedg_mesh m, T* M, hipStream_t stream) {
  switch (m->b) {
    case 1: return factor_levels_small<T, 1>(ctx, m, M, stream);
    case 2: return factor_levels_small<T, 2>(ctx, m, M, stream);
    case 3: return factor_levels_small<T, 3>(ctx, m, M, stream);
    case 4: return factor_levels_small<T, 4>(ctx, m, M, stream);
    case 5: return factor_levels_small<T, 5>(ctx, m, M, stream);
    case 6: return factor_levels_small<T, 6>(ctx, m, M, stream);
    case 7: return factor_levels_small<T, 7>(ctx, m, M, stream);
    case 8: return factor_levels_small<T, 8>(ctx, m, M, stream);
    default: break;
  }
  switch ((m->b + 15) / 16) {
    case 1: return factor_levels_nb<T, 1>(ctx, m, M, stream);
    case 2: return factor_levels_nb<T, 2>(ctx, m, M, stream);
    case 3: return factor_levels_nb<T, 3>(ctx, m, M, stream);
    case 4: return factor_levels_nb<T, 4>(ctx, m, M, stream);
    case 5: return factor_levels_nb<T, 5>(ctx, m, M, stream);
    case 6: return factor_levels_nb<T, 6>(ctx, m, M, stream);
    case 7: return factor_levels_nb<T, 7>(ctx, m, M, stream);
    case 8: return factor_levels_nb<T, 8>(ctx, m, M, stream);
  }
  return set_error(ctx, IEDG_ERR_UNSUPPORTED, "factor_ilu0: b=%d", m->b);
}

extern "C" {

iedg_status iedg_assemble(iedg_context ctx, iedg_mesh m, iedg_prec prec, const void* Ke, const double* r,
                          const double* G, void* Kbsr, double* R, hipStream_t stream) {
  if (!ctx || !m) return IEDG_ERR_INVALID_ARG;
  if ((Ke == nullptr) != (Kbsr == nullptr)) return set_error(ctx, IEDG_ERR_INVALID_ARG, "assemble: Ke and Kbsr go together");
  if ((r || G) && !R) return set_error(ctx, IEDG_ERR_INVALID_ARG, "assemble: R missing");
  if (prec != IEDG_F64 && prec != IEDG_F32 && prec != IEDG_BF16)
    return set_error(ctx, IEDG_ERR_INVALID_ARG, "assemble: precision");
  if (Ke) {
    if (m->b < 16) {
      const int64_t total = m->nnzb * m->b * m->b;
      const unsigned grid = (unsigned)((total + 255) / 256);
      if (prec == IEDG_F64)
        hipLaunchKernelGGL(assemble_k_small_kernel<double>, dim3(grid), dim3(256), 0, stream, m->b, m->t, m->slots,
                           m->nnzb, m->d_asm_ptr, m->d_asm_list, (const double*)Ke, (double*)Kbsr);
      else
        hipLaunchKernelGGL(assemble_k_small_kernel<float>, dim3(grid), dim3(256), 0, stream, m->b, m->t, m->slots,
                           m->nnzb, m->d_asm_ptr, m->d_asm_list, (const float*)Ke, (float*)Kbsr);
    } else {
      const size_t smem = prec_size(prec) * m->b * (m->b + 1);
      if (prec == IEDG_F64) {
        auto k = assemble_k_kernel<double>;
        IEDG_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
        hipLaunchKernelGGL(k, dim3(m->nnzb), dim3(STHR), smem, stream, m->b, m->t, m->slots, m->d_asm_ptr,
                           m->d_asm_list, (const double*)Ke, (double*)Kbsr);
      } else {
        auto k = assemble_k_kernel<float>;
        IEDG_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
        hipLaunchKernelGGL(k, dim3(m->nnzb), dim3(STHR), smem, stream, m->b, m->t, m->slots, m->d_asm_ptr,
                           m->d_asm_list, (const float*)Ke, (float*)Kbsr);
      }
    }
    IEDG_LAUNCH_CHECK(ctx, "assemble K launch");
  }
  if (R) {
    const int64_t total = m->n_trace;
    hipLaunchKernelGGL(assemble_r_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, m->n_face,
                       m->b, m->t, m->slots, m->d_src_ptr, m->d_src_list, r, G, R);
    IEDG_LAUNCH_CHECK(ctx, "assemble R launch");
  }
  return IEDG_OK;
}

iedg_status iedg_factor_ilu0(iedg_context ctx, iedg_mesh m, iedg_prec prec, const void* Kbsr, void* Mbsr,
                             hipStream_t stream) {
  if (!ctx || !m || !Kbsr || !Mbsr) return IEDG_ERR_INVALID_ARG;
  if (prec != IEDG_F64 && prec != IEDG_F32 && prec != IEDG_BF16)
    return set_error(ctx, IEDG_ERR_UNSUPPORTED, "factor_ilu0: precision");
  const size_t es = prec_size(prec);
  if (Kbsr != Mbsr)
    IEDG_HIP(ctx, hipMemcpyAsync(Mbsr, Kbsr, es * m->nnzb * m->b * m->b, hipMemcpyDeviceToDevice, stream));
  if (prec == IEDG_F64) return factor_levels<double>(ctx, m, (double*)Mbsr, stream);
  return factor_levels<float>(ctx, m, (float*)Mbsr, stream);
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
