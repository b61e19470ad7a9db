// Element static condensation on gfx950 (section 2.2.1, eq. LS).
//
// Per element the bordered matrix  M = [A B F; C D 0]  (N = n + t rows,
// NC = N + 1 columns with F) is reduced by n steps of Gaussian elimination
// with partial pivoting over the rows of A.  After those steps
//   rows < n :  unit-lower L and U of P A, U12 = L^{-1} P B, w = L^{-1} P F
//   rows >= n:  L21 = C U^{-1},  Ke = D - L21 U12,  r = -L21 w
// so the trailing block is the Schur complement D - C A^{-1} B of eq. LS.
//
// Schedule (one 256-thread workgroup per element, 64-wide panels):
//   for each panel [c0, c1):
//     1. panel column, Crout order: M[c0:, c0:c1] -= L[c0:, :c0] U[:c0, c0:c1]
//        (FP64/FP32 MFMA tiles reading the already factored parts)
//     2. panel factorisation: 8-column leaves held in registers, partial
//        pivoting over rows c0..n-1 with a workgroup argmax per column,
//        rows of C finished by a triangular solve with the leaf's U
//     3. panel row: U[c0:c1, c1:] = L_pp^{-1} (M[c0:c1, c1:] - L[c0:c1,:c0] U[:c0, c1:])
//   4. Schur block: M[n:, n:] -= L21 U12 (MFMA, K = n)
// Every entry of M is read from the inputs exactly once, when its tile is
// first formed; row interchanges of not-yet-read rows are carried by a
// permutation in LDS, those of already written L rows are applied in place.
#include <climits>

#include "common.h"

namespace iedg {

constexpr int CT = 64;        // Crout tile / panel width
constexpr int CTP = CT + 1;   // padded LDS row stride
constexpr int CTHR = 256;     // threads per workgroup (4 waves)
constexpr int LW = 8;         // leaf width of the panel factorisation

template <typename T>
struct CondenseArgs {
  int E, n, t;
  const double *A, *B, *C, *D, *F;
  T *LU, *U12, *L21, *Ke;
  int32_t* perm;
  double *w, *r;
  DeviceStatus* status;
};

// Addressing of one element's bordered matrix (inputs and outputs).
template <typename T>
struct Elem {
  int n, t, N, NC;
  const double *A, *B, *C, *D, *F;
  T *LU, *U12, *L21, *Ke;
  double *w, *r;
  const int* sperm;

  __device__ T in(int row, int col) const {
    if (row < n) {
      const size_t pr = (size_t)sperm[row];
      if (col < n) return (T)A[pr * n + col];
      if (col < N) return (T)B[pr * t + (col - n)];
      return (T)F[pr];
    }
    const size_t q = (size_t)(row - n);
    if (col < n) return (T)C[q * n + col];
    if (col < N) return (T)D[q * t + (col - n)];
    return T(0);
  }
  __device__ T ld(int row, int col) const {
    if (row < n) {
      if (col < n) return LU[(size_t)row * n + col];
      if (col < N) return U12[(size_t)row * t + (col - n)];
      return (T)w[row];
    }
    const size_t q = (size_t)(row - n);
    if (col < n) return L21[q * n + col];
    if (col < N) return Ke[q * t + (col - n)];
    return (T)r[q];
  }
  __device__ void st(int row, int col, T v) const {
    if (row < n) {
      if (col < n) LU[(size_t)row * n + col] = v;
      else if (col < N) U12[(size_t)row * t + (col - n)] = v;
      else w[row] = (double)v;
      return;
    }
    const size_t q = (size_t)(row - n);
    if (col < n) L21[q * n + col] = v;
    else if (col < N) Ke[q * t + (col - n)] = v;
    else r[q] = (double)v;
  }
  // row `row` of the L part (columns < n)
  __device__ const T* lrow(int row) const {
    return row < n ? LU + (size_t)row * n : L21 + (size_t)(row - n) * n;
  }
};

template <typename T>
__device__ inline void load4(const T* p, T (&v)[4]);
template <>
__device__ inline void load4<double>(const double* p, double (&v)[4]) {
  const double2 a = *reinterpret_cast<const double2*>(p);
  const double2 b = *reinterpret_cast<const double2*>(p + 2);
  v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
template <>
__device__ inline void load4<float>(const float* p, float (&v)[4]) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}

// acc = L[rows, 0:K] * U[0:K, cols] for this wave's 32x32 quadrant of the
// 64x64 tile at (r0, c0); rows >= rlim and cols >= clim read as zero.
template <typename T>
__device__ void tile_gemm(const Elem<T>& el, int r0, int rlim, int c0, int clim, int K,
                          typename Mfma<T>::acc_t (&acc)[2][2]) {
  typedef Mfma<T> MF;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int rq = r0 + 32 * (wv >> 1), cq = c0 + 32 * (wv & 1);
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = MF::zero();
  if (K <= 0) return;
  const T* arow[2];
  bool aok[2];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb) {
    const int row = rq + 16 * rb + li;
    aok[rb] = row < rlim;
    arow[rb] = el.lrow(aok[rb] ? row : 0);
  }
  // B operand: column `col` of the U part (LU upper, U12 or w)
  const T* bbase[2];
  const double* wbase[2];
  int bstride[2];
  bool bok[2];
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    const int col = cq + 16 * cb + li;
    bok[cb] = col < clim;
    wbase[cb] = nullptr;
    if (col < el.n) { bbase[cb] = el.LU + col; bstride[cb] = el.n; }
    else if (col < el.N) { bbase[cb] = el.U12 + (col - el.n); bstride[cb] = el.t; }
    else { bbase[cb] = el.LU; bstride[cb] = 1; wbase[cb] = el.w; }
  }
  T a[2][4], b[2][4], an[2][4], bn[2][4];
  auto load = [&](int k0, T (&ao)[2][4], T (&bo)[2][4]) {
    const int kb = k0 + 4 * lk;
    const bool full = kb + 3 < K;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      if (aok[rb] && full) {
        load4<T>(arow[rb] + kb, ao[rb]);
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) ao[rb][s] = (aok[rb] && kb + s < K) ? arow[rb][kb + s] : T(0);
      }
    }
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = kb + s;
        T v = T(0);
        if (bok[cb] && k < K) v = wbase[cb] ? (T)wbase[cb][k] : bbase[cb][(size_t)k * bstride[cb]];
        bo[cb][s] = v;
      }
    }
  };
  load(0, a, b);
  for (int k0 = 0; k0 < K; k0 += 16) {
    const bool more = k0 + 16 < K;
    if (more) load(k0 + 16, an, bn);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = MF::mac(a[rb][s], b[cb][s], acc[rb][cb]);
    if (more) {
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int s = 0; s < 4; ++s) { a[rb][s] = an[rb][s]; b[rb][s] = bn[rb][s]; }
    }
  }
}

// For each accumulator element of this wave: (row, col) inside the tile.
template <typename T, typename F>
__device__ inline void for_acc(int r0, int c0, typename Mfma<T>::acc_t (&acc)[2][2], F f) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int rq = r0 + 32 * (wv >> 1), cq = c0 + 32 * (wv & 1);
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        f(rq + 16 * rb + Mfma<T>::row(lane, v), cq + 16 * cb + (lane & 15), acc[rb][cb][v]);
}

struct LeafSmem {
  double red_v[4];
  int red_i[4];
  int swaps[LW];
};

// Factor panel columns [c0, c1) (already Crout-updated) in leaves of LW.
template <typename T, int QMAX, int QCMAX, int LWT>
__device__ void panel_factor(const Elem<T>& el, int* sperm, int c0, int c1, T* sprow, T* skrow,
                             T* suleaf, T* slleaf, T* sU, LeafSmem* ls, DeviceStatus* status, int elem) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n = el.n, N = el.N;
  for (int cs = c0; cs < c1; cs += LWT) {
    const int ce = min(cs + LWT, c1), lw = ce - cs;
    T x[QMAX][LWT];
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const int row = cs + tid + CTHR * q;
#pragma unroll
      for (int j = 0; j < LWT; ++j) x[q][j] = (row < n && j < lw) ? el.ld(row, cs + j) : T(0);
    }
#pragma unroll
    for (int kk = 0; kk < LWT; ++kk) {
      if (kk < lw) {
        const int k = cs + kk;
        double best = -1.0;
        int bidx = INT_MAX;
#pragma unroll
        for (int q = 0; q < QMAX; ++q) {
          const int row = cs + tid + CTHR * q;
          const double v = fabs((double)x[q][kk]);
          if (row >= k && row < n && (v > best)) { best = v; bidx = row; }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          const double ov = __shfl_xor(best, off, kWave);
          const int oi = __shfl_xor(bidx, off, kWave);
          if (ov > best || (ov == best && oi < bidx)) { best = ov; bidx = oi; }
        }
        if (lane == 0) { ls->red_v[wv] = best; ls->red_i[wv] = bidx; }
        __syncthreads();
        best = ls->red_v[0];
        bidx = ls->red_i[0];
#pragma unroll
        for (int i = 1; i < 4; ++i) {
          const double ov = ls->red_v[i];
          const int oi = ls->red_i[i];
          if (ov > best || (ov == best && oi < bidx)) { best = ov; bidx = oi; }
        }
        int piv = bidx;
        if (piv == INT_MAX || !(best > 0.0) || !isfinite(best)) {
          if (tid == 0) latch_status(status, IEDG_ERR_SINGULAR, elem);
          piv = k;
        }
        const int po = piv - cs;  // owner of the pivot row: tid po % CTHR, slot po / CTHR
        if (tid == (po % CTHR)) {
#pragma unroll
          for (int q = 0; q < QMAX; ++q)
            if (q == po / CTHR)
#pragma unroll
              for (int j = 0; j < LWT; ++j) sprow[j] = x[q][j];
        }
        if (tid == kk) {
#pragma unroll
          for (int j = 0; j < LWT; ++j) skrow[j] = x[0][j];
        }
        __syncthreads();
        if (piv != k && tid == (po % CTHR)) {
#pragma unroll
          for (int q = 0; q < QMAX; ++q)
            if (q == po / CTHR)
#pragma unroll
              for (int j = 0; j < LWT; ++j) x[q][j] = skrow[j];
        }
        if (tid == kk) {
#pragma unroll
          for (int j = 0; j < LWT; ++j) x[0][j] = sprow[j];
        }
        if (tid == 0) {
          const int tmp = sperm[k];
          sperm[k] = sperm[piv];
          sperm[piv] = tmp;
          ls->swaps[kk] = piv;
        }
        if (tid < LWT) suleaf[kk * LW + tid] = sprow[tid];
        const T ukk = sprow[kk];
        T u[LWT];
#pragma unroll
        for (int j = 0; j < LWT; ++j) u[j] = sprow[j];
#pragma unroll
        for (int q = 0; q < QMAX; ++q) {
          const int row = cs + tid + CTHR * q;
          if (row > k && row < n) {
            const T l = x[q][kk] / ukk;
            x[q][kk] = l;
#pragma unroll
            for (int j = kk + 1; j < LWT; ++j) x[q][j] -= l * u[j];
          }
        }
        __syncthreads();
      }
    }
    // write the leaf back (rows of A) and record L of the leaf's own rows
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const int row = cs + tid + CTHR * q;
      if (row < n)
#pragma unroll
        for (int j = 0; j < LWT; ++j)
          if (j < lw) el.st(row, cs + j, x[q][j]);
    }
    if (tid < lw) {
#pragma unroll
      for (int j = 0; j < LWT; ++j) slleaf[tid * LW + j] = (j < tid) ? x[0][j] : T(0);
    }
    // rows of C: L21 = X U_leaf^{-1}
    T xc[QCMAX][LWT];
#pragma unroll
    for (int q = 0; q < QCMAX; ++q) {
      const int row = n + tid + CTHR * q;
      const bool ok = row < N;
#pragma unroll
      for (int j = 0; j < LWT; ++j) xc[q][j] = (ok && j < lw) ? el.ld(row, cs + j) : T(0);
      if (ok) {
#pragma unroll
        for (int j = 0; j < LWT; ++j) {
          if (j < lw) {
            T v = xc[q][j];
#pragma unroll
            for (int k2 = 0; k2 < j; ++k2) v -= xc[q][k2] * suleaf[k2 * LW + j];
            xc[q][j] = v / suleaf[j * LW + j];
            el.st(row, cs + j, xc[q][j]);
          }
        }
      }
    }
    // apply this leaf's interchanges to the columns outside the leaf that
    // hold already-formed values: [0, cs) (L) and [ce, c1) (panel remainder)
    {
      const int nother = cs + (c1 - ce);
      for (int m = tid; m < nother; m += CTHR) {
        const int col = m < cs ? m : ce + (m - cs);
        for (int kk = 0; kk < lw; ++kk) {
          const int p = ls->swaps[kk];
          const int k = cs + kk;
          if (p != k) {
            const T a = el.ld(k, col), b2 = el.ld(p, col);
            el.st(k, col, b2);
            el.st(p, col, a);
          }
        }
      }
    }
    __syncthreads();
    const int nright = c1 - ce;
    if (nright > 0) {
      // (i) rows [cs, ce) of the remaining panel columns: U = L_leaf^{-1} X
      if (tid < nright) {
        const int col = ce + tid;
        T v[LWT];
#pragma unroll
        for (int i = 0; i < LWT; ++i) {
          if (i < lw) {
            T s = el.ld(cs + i, col);
#pragma unroll
            for (int k2 = 0; k2 < i; ++k2) s -= slleaf[i * LW + k2] * v[k2];
            v[i] = s;
            el.st(cs + i, col, s);
            sU[i * CT + tid] = s;
          } else {
            v[i] = T(0);
            sU[i * CT + tid] = T(0);
          }
        }
      }
      __syncthreads();
      // (ii) rank-lw update of rows [ce, N) in the remaining panel columns
#pragma unroll
      for (int q = 0; q < QMAX; ++q) {
        const int row = cs + tid + CTHR * q;
        if (row >= ce && row < n) {
          for (int j = 0; j < nright; ++j) {
            T s = el.ld(row, ce + j);
#pragma unroll
            for (int k2 = 0; k2 < LWT; ++k2) s -= x[q][k2] * sU[k2 * CT + j];
            el.st(row, ce + j, s);
          }
        }
      }
#pragma unroll
      for (int q = 0; q < QCMAX; ++q) {
        const int row = n + tid + CTHR * q;
        if (row < N) {
          for (int j = 0; j < nright; ++j) {
            T s = el.ld(row, ce + j);
#pragma unroll
            for (int k2 = 0; k2 < LWT; ++k2) s -= xc[q][k2] * sU[k2 * CT + j];
            el.st(row, ce + j, s);
          }
        }
      }
    }
    __syncthreads();
  }
}

template <typename T, int QMAX, int QCMAX, int LWT>
__global__ __launch_bounds__(CTHR) void condense_kernel(CondenseArgs<T> a) {
  typedef Mfma<T> MF;
  const int e = blockIdx.x;
  const int tid = threadIdx.x;
  const int n = a.n, t = a.t, N = n + t;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sLinv = reinterpret_cast<T*>(smem_raw);          // CT x CTP
  T* sX = sLinv + CT * CTP;                           // CT x CTP
  T* sprow = sX + CT * CTP;                           // LW
  T* skrow = sprow + LW;                              // LW
  T* suleaf = skrow + LW;                             // LW x LW
  T* slleaf = suleaf + LW * LW;                       // LW x LW
  T* sU = slleaf + LW * LW;                           // LW x CT
  LeafSmem* ls = reinterpret_cast<LeafSmem*>(sU + LW * CT);
  int* sperm = reinterpret_cast<int*>(ls + 1);        // n

  Elem<T> el;
  el.n = n; el.t = t; el.N = N; el.NC = a.F ? N + 1 : N;
  const size_t nn = (size_t)n * n, nt = (size_t)n * t, tt = (size_t)t * t;
  el.A = a.A + e * nn; el.B = a.B + e * nt; el.C = a.C + e * nt; el.D = a.D + e * tt;
  el.F = a.F ? a.F + (size_t)e * n : nullptr;
  el.LU = a.LU + e * nn; el.U12 = a.U12 + e * nt; el.L21 = a.L21 + e * nt; el.Ke = a.Ke + e * tt;
  el.w = a.w ? a.w + (size_t)e * n : nullptr;
  el.r = a.r ? a.r + (size_t)e * t : nullptr;
  el.sperm = sperm;
  const int NC = el.NC;

  for (int i = tid; i < n; i += CTHR) sperm[i] = i;
  __syncthreads();

  typename MF::acc_t acc[2][2];
  for (int c0 = 0; c0 < n; c0 += CT) {
    const int c1 = min(c0 + CT, n);
    // 1. panel column in Crout order
    for (int r0 = c0; r0 < N; r0 += CT) {
      tile_gemm<T>(el, r0, N, c0, c1, c0, acc);
      for_acc<T>(r0, c0, acc, [&](int row, int col, T v) {
        if (row < N && col < c1) el.st(row, col, el.in(row, col) - v);
      });
    }
    __syncthreads();
    // 2. factor the panel
    panel_factor<T, QMAX, QCMAX, LWT>(el, sperm, c0, c1, sprow, skrow, suleaf, slleaf, sU, ls, a.status, e);
    // 3a. L_pp^{-1} (unit lower, zero padded) into sLinv
    const int wp = c1 - c0;
    for (int i = tid; i < CT * CT; i += CTHR) {
      const int r = i / CT, c = i % CT;
      sX[r * CTP + c] = (r < wp && c < r) ? el.ld(c0 + r, c0 + c) : T(0);
    }
    __syncthreads();
    if (tid < CT) {
      const int j = tid;
      for (int i = 0; i < CT; ++i) {
        T s = (i == j) ? T(1) : T(0);
        if (i > j && i < wp) {
          for (int k = j; k < i; ++k) s -= sX[i * CTP + k] * sLinv[k * CTP + j];
        }
        sLinv[i * CTP + j] = (i < wp && j < wp) ? s : T(0);
      }
    }
    __syncthreads();
    // 3b. panel row: U[c0:c1, c1:NC]
    for (int j0 = c1; j0 < NC; j0 += CT) {
      const int jl = min(j0 + CT, NC);
      tile_gemm<T>(el, c0, c1, j0, jl, c0, acc);
      for_acc<T>(c0, j0, acc, [&](int row, int col, T v) {
        sX[(row - c0) * CTP + (col - j0)] = (row < c1 && col < jl) ? el.in(row, col) - v : T(0);
      });
      __syncthreads();
      // acc = Linv (64x64) * X (64x64) from LDS
      {
        const int lane = tid & 63, wv = tid >> 6;
        const int li = lane & 15, lk = lane >> 4;
        const int rq = 32 * (wv >> 1), cq = 32 * (wv & 1);
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
          for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = MF::zero();
        for (int k0 = 0; k0 < wp; k0 += 4) {
          T av[2], bv[2];
#pragma unroll
          for (int rb = 0; rb < 2; ++rb) av[rb] = sLinv[(rq + 16 * rb + li) * CTP + k0 + lk];
#pragma unroll
          for (int cb = 0; cb < 2; ++cb) bv[cb] = sX[(k0 + lk) * CTP + cq + 16 * cb + li];
#pragma unroll
          for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = MF::mac(av[rb], bv[cb], acc[rb][cb]);
        }
      }
      for_acc<T>(c0, j0, acc, [&](int row, int col, T v) {
        if (row < c1 && col < jl) el.st(row, col, v);
      });
      __syncthreads();
    }
    __syncthreads();
  }
  // 4. Schur block
  for (int r0 = n; r0 < N; r0 += CT) {
    for (int j0 = n; j0 < NC; j0 += CT) {
      const int jl = min(j0 + CT, NC);
      tile_gemm<T>(el, r0, N, j0, jl, n, acc);
      for_acc<T>(r0, j0, acc, [&](int row, int col, T v) {
        if (row < N && col < jl) el.st(row, col, el.in(row, col) - v);
      });
    }
  }
  for (int i = tid; i < n; i += CTHR) a.perm[(size_t)e * n + i] = sperm[i];
}

template <typename T>
static size_t condense_smem(int n) {
  return sizeof(T) * (2 * CT * CTP + 2 * LW + 2 * LW * LW + LW * CT) + sizeof(LeafSmem) + sizeof(int) * n;
}

template <typename T, int QMAX, int QCMAX, int LWT>
static hipError_t launch_condense(const CondenseArgs<T>& a, hipStream_t s) {
  const size_t smem = condense_smem<T>(a.n);
  auto kern = condense_kernel<T, QMAX, QCMAX, LWT>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(a.E), dim3(CTHR), smem, s, a);
  return hipGetLastError();
}

template <typename T>
static hipError_t dispatch_condense(const CondenseArgs<T>& a, hipStream_t s) {
  const int qa = (a.n + CTHR - 1) / CTHR, qc = (a.t + CTHR - 1) / CTHR;
  if (qa <= 3 && qc <= 2) return launch_condense<T, 3, 2, 8>(a, s);
  if (qa <= 5 && qc <= 2) return launch_condense<T, 5, 2, 8>(a, s);
  if (qa <= 10 && qc <= 3) return launch_condense<T, 10, 3, 4>(a, s);
  return hipErrorInvalidValue;
}

// ---- right-hand side condensation: w = L^{-1} P F, r = -L21 w ----------
constexpr int RTHR = 256;

template <typename T>
__global__ __launch_bounds__(RTHR) void condense_rhs_kernel(int n, int t, const T* LU, const int32_t* perm,
                                                            const T* L21, const double* F, double* w,
                                                            double* r) {
  const int e = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* y = reinterpret_cast<double*>(smem_raw);  // n
  double* blk = y + n;                              // 64 x 65
  const T* L = LU + (size_t)e * n * n;
  const int32_t* p = perm + (size_t)e * n;
  const double* f = F + (size_t)e * n;
  for (int i = tid; i < n; i += RTHR) y[i] = f[p[i]];
  __syncthreads();
  for (int i0 = 0; i0 < n; i0 += 64) {
    const int i1 = min(i0 + 64, n), bw = i1 - i0;
    // y[i0:i1] -= L[i0:i1, 0:i0] y[0:i0]   (one wave per row)
    for (int i = i0 + wv; i < i1; i += RTHR / 64) {
      double s = 0.0;
      const T* row = L + (size_t)i * n;
      for (int k = lane; k < i0; k += 64) s += (double)row[k] * y[k];
      s = wave_sum(s);
      if (lane == 0) y[i] -= s;
    }
    for (int q = tid; q < 64 * 64; q += RTHR) {
      const int rr = q / 64, cc = q % 64;
      blk[rr * 65 + cc] = (rr < bw && cc < rr) ? (double)L[(size_t)(i0 + rr) * n + i0 + cc] : 0.0;
    }
    __syncthreads();
    if (wv == 0) {
      double yl = lane < bw ? y[i0 + lane] : 0.0;
      for (int k = 0; k < bw; ++k) {
        const double yk = __shfl(yl, k, kWave);
        if (lane > k) yl -= blk[lane * 65 + k] * yk;
      }
      if (lane < bw) y[i0 + lane] = yl;
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += RTHR) w[(size_t)e * n + i] = y[i];
  const T* L2 = L21 + (size_t)e * t * n;
  for (int i = wv; i < t; i += RTHR / 64) {
    double s = 0.0;
    const T* row = L2 + (size_t)i * n;
    for (int k = lane; k < n; k += 64) s += (double)row[k] * y[k];
    s = wave_sum(s);
    if (lane == 0) r[(size_t)e * t + i] = -s;
  }
}

}  // namespace iedg

using namespace iedg;

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
  if (n_local > 10 * CTHR || n_trace_elem > 3 * CTHR)
    return set_error(ctx, IEDG_ERR_UNSUPPORTED, "condense: n=%d t=%d too large", n_local, n_trace_elem);
  hipError_t err;
  if (prec == IEDG_F64) {
    CondenseArgs<double> a{n_elem, n_local, n_trace_elem, A, B, C, D, F,
                           (double*)LU, (double*)U12, (double*)L21, (double*)Ke, perm, w, r, ctx->d_status};
    err = dispatch_condense<double>(a, stream);
  } else if (prec == IEDG_F32) {
    CondenseArgs<float> a{n_elem, n_local, n_trace_elem, A, B, C, D, F,
                          (float*)LU, (float*)U12, (float*)L21, (float*)Ke, perm, w, r, ctx->d_status};
    err = dispatch_condense<float>(a, stream);
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
  const size_t smem = sizeof(double) * (n_local + 64 * 65);
  if (prec == IEDG_F64) {
    auto k = condense_rhs_kernel<double>;
    IEDG_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
    hipLaunchKernelGGL(k, dim3(n_elem), dim3(RTHR), smem, stream, n_local, n_trace_elem, (const double*)LU, perm,
                       (const double*)L21, F, w, r);
  } else if (prec == IEDG_F32 || prec == IEDG_BF16) {
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
