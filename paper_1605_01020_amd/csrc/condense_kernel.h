#pragma once
// Element static condensation on gfx950 (section 2.2.1, eq. LS): the kernel.
// Included by two translation units per precision (condense_<p>.hip: the
// persistent batched form; condense_<p>_single.hip: one element per
// workgroup), so they compile in parallel.
//
// Per element the bordered matrix  M = [A B F; C D 0]  (N = n + t rows,
// NC = N + 1 columns with F) is reduced by n steps of Gaussian elimination
// with partial pivoting over the rows of A.  After those steps
//   rows of A:  unit-lower L and U of P A, U12 = L^{-1} P B, w = L^{-1} P F
//   rows of C:  L21 = C U^{-1},  Ke = D - L21 U12,  r = -L21 w
// so the trailing block is the Schur complement D - C A^{-1} B of eq. LS.
//
// Row interchanges never move data: pivot position i of P A lives in the
// physical row perm[i] of every A-row-indexed array (A itself, LU, U12, w),
// and only the permutation in LDS is updated when a pivot is chosen.
//
// Schedule, one 512-thread workgroup (8 waves) per element, panels of CT =
// 64 or (FP32 storage) 128 columns:
//   for each panel [c0, c1):
//     1. panel column (Crout order): M[c0:, c0:c1] = in - L[c0:, :c0] U[:c0, c0:c1]
//        -- MFMA tiles of 256 x CT fed from double-buffered LDS k-slabs
//     2. panel factorisation in register-resident sub-panels of 16 (or 8)
//        columns: each sub-panel first takes the updates of the panel's
//        earlier sub-panels (left-looking), then partial pivoting with one
//        workgroup barrier per column; the panel's L^{-1} is grown in LDS
//        (a 128-wide panel in two halves of 64 with one MFMA update between)
//     3. panel row: U[c0:c1, c1:] = L_pp^{-1} (in - L[c0:c1, :c0] U[:c0, c1:])
//        -- MFMA tiles of CT x 256; the triangular solve with L_pp^{-1} is a
//        second MFMA pass on the accumulators (each wave owns whole columns)
//   4. Schur block: M[n:, n:] = in - L21 U12 (MFMA, K = n)
// BF16 operand mode: the GEMM operands are rounded to BF16 once, as they
// enter the LDS slab; accumulation, panels and storage stay FP32.
#include <algorithm>
#include <climits>

#include "common.h"
#include "condense.h"

namespace iedg {

// Wave-wide maximum and minimum without a round trip through LDS: two quad
// permutations and two rotations inside each 16-lane row (DPP) leave the
// row's extremum in every lane of the row; the four rows are then read as
// uniform values.  The result is the same in every lane.
constexpr int kDppXor1 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;   // quad_perm [2,3,0,1]
constexpr int kDppRor4 = 0x124;  // row_ror:4
constexpr int kDppRor8 = 0x128;  // row_ror:8

template <int CTRL>
__device__ __attribute__((always_inline)) inline int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __attribute__((always_inline)) inline float dpp_move(float v) {
  return __int_as_float(dpp_i32<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __attribute__((always_inline)) inline double dpp_move(double v) {
  return __hiloint2double(dpp_i32<CTRL>(__double2hiint(v)), dpp_i32<CTRL>(__double2loint(v)));
}
template <int CTRL>
__device__ __attribute__((always_inline)) inline int dpp_move(int v) {
  return dpp_i32<CTRL>(v);
}
__device__ __attribute__((always_inline)) inline float read_lane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __attribute__((always_inline)) inline double read_lane(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
__device__ __attribute__((always_inline)) inline int read_lane(int v, int l) {
  return __builtin_amdgcn_readlane(v, l);
}

// (values must not be NaN)
template <typename T>
__device__ __attribute__((always_inline)) inline T wave_max(T v) {
  v = fmax(v, dpp_move<kDppXor1>(v));
  v = fmax(v, dpp_move<kDppXor2>(v));
  v = fmax(v, dpp_move<kDppRor4>(v));
  v = fmax(v, dpp_move<kDppRor8>(v));
  return fmax(fmax(read_lane(v, 0), read_lane(v, 16)), fmax(read_lane(v, 32), read_lane(v, 48)));
}
__device__ __attribute__((always_inline)) inline int wave_min(int v) {
  v = min(v, dpp_move<kDppXor1>(v));
  v = min(v, dpp_move<kDppXor2>(v));
  v = min(v, dpp_move<kDppRor4>(v));
  v = min(v, dpp_move<kDppRor8>(v));
  return min(min(read_lane(v, 0), read_lane(v, 16)), min(read_lane(v, 32), read_lane(v, 48)));
}


constexpr int NT = 512;       // threads per workgroup (8 waves)
static_assert(NT == 512, "default_leaf_width counts rows per thread for 512 threads");
constexpr int NW = NT / 64;   // waves
constexpr int SWMAX = 16;     // widest sub-panel (LDS sizing)
constexpr int KC = 16;        // k-slab depth of the GEMM engine
// Panel width CT (64 or 128 columns; 128 only in FP32 storage, whose panel
// buffers fit the LDS at that width) with the tile shapes of the GEMM phases
// (rows x columns): panel columns CM x CT, panel rows CT x RN (waves stacked
// along columns: the triangular solve on the accumulators needs all CT rows
// in each wave), Schur block SM x SN.  CT = 64: 256 x 64, 64 x 256, 256 x 64;
// CT = 128: 256 x 128, 128 x 256, 256 x 128 (64 accumulators a lane in
// every shape).  Wider panels halve the re-reads of the L and U operands
// that the Crout updates stream from HBM, and 256-row tiles read the
// right-hand operand once for 256 rows instead of 128; narrow elements
// factor faster in narrow panels (the width is tuned per element size).
template <typename T, int CT>
struct Shapes {
  static_assert(CT == 64 || (CT == 128 && sizeof(T) == 4), "panel width");
  static constexpr int LIS = CT + 1;  // LDS stride of L^{-1}
  static constexpr bool W = CT == 128;
  static constexpr int CM = 256;
  static constexpr int RN = 256;
  static constexpr int SM = 256, SN = W ? 128 : 64;
};
// The widest panel a precision is built for.
template <typename T>
constexpr int CT_MAX = sizeof(T) == 4 ? 128 : 64;



// Addressing of one element's bordered matrix.  Rows are pivot positions;
// a position p < n lives in physical row sperm[p] of A, B, F, LU, U12, w.
template <typename T>
struct Elem {
  int n, t, N, NC;
  const double *A, *B, *C, *D, *F;
  T *LU, *U12, *L21, *Ke;
  double *w, *r;
  const int* sperm;

  // Input value at (row, col).  FP32 storage: A, B, C, D were first copied
  // (converted) into the output arrays, whose entries are read exactly once
  // as input before they are overwritten (Crout order), so the input is read
  // there in the storage type -- no conversion stands between the load and
  // the MFMA accumulators it initialises.
  __device__ __attribute__((always_inline)) T in(int row, int col) const {
    if constexpr (sizeof(T) == 4) {
      if (col < N) return ld(row, col);
      return row < n ? (T)F[sperm[row]] : T(0);
    } else {
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
  }
  __device__ __attribute__((always_inline)) T ld(int row, int col) const {
    if (row < n) {
      const size_t pr = (size_t)sperm[row];
      if (col < n) return LU[pr * n + col];
      if (col < N) return U12[pr * t + (col - n)];
      return (T)w[pr];
    }
    const size_t q = (size_t)(row - n);
    if (col < n) return L21[q * n + col];
    if (col < N) return Ke[q * t + (col - n)];
    return (T)r[q];
  }
  __device__ __attribute__((always_inline)) void st(int row, int col, T v) const {
    if (row < n) {
      const size_t pr = (size_t)sperm[row];
      if (col < n) LU[pr * n + col] = v;
      else if (col < N) U12[pr * t + (col - n)] = v;
      else w[pr] = (double)v;
      return;
    }
    const size_t q = (size_t)(row - n);
    if (col < n) L21[q * n + col] = v;
    else if (col < N) Ke[q * t + (col - n)] = v;
    else r[q] = (double)v;
  }
  // L part (columns < n) of position `row`
  __device__ __attribute__((always_inline)) T* lrow(int row) const {
    return row < n ? LU + (size_t)sperm[row] * n : L21 + (size_t)(row - n) * n;
  }
  // One column segment of position `row` (SEG 0: columns [0, n), SEG 1:
  // columns [n, N)), indexed by col - seg_base<SEG>(): the same entries as
  // st() and in() reach, with the row resolved once for all its columns.
  template <int SEG>
  __device__ __attribute__((always_inline)) int seg_base() const { return SEG ? n : 0; }
  template <int SEG>
  __device__ __attribute__((always_inline)) T* out_row(int row) const {
    if constexpr (SEG == 0) return lrow(row);
    return row < n ? U12 + (size_t)sperm[row] * t : Ke + (size_t)(row - n) * t;
  }
  template <int SEG>
  __device__ __attribute__((always_inline)) const T* in_row(int row) const {
    if constexpr (sizeof(T) == 4) {
      return out_row<SEG>(row);  // FP32: inputs were copied into the outputs
    } else if constexpr (SEG == 0) {
      return row < n ? A + (size_t)sperm[row] * n : C + (size_t)(row - n) * n;
    } else {
      return row < n ? B + (size_t)sperm[row] * t : D + (size_t)(row - n) * t;
    }
  }
};

template <typename T> struct Pair;
template <> struct Pair<double> { typedef double2 v; };
template <> struct Pair<float> { typedef float2 v; };

// ---- GEMM engine ----------------------------------------------------------
// acc = in - L[r0:r0+TM, 0:K] * U[0:K, c0:c0+TN] for the workgroup's TM x TN
// tile (in = the bordered matrix's input values); rows >= rlim, cols >= clim
// and k >= K read as zero.  Waves are stacked along rows (256 x 64: each
// wave 32 x 64; 256 x 128: 32 x 128) or, with COLS (the default for wide
// tiles), along columns (64 x 256: 64 x 32; 128 x 256: 128 x 32).  k-slabs
// of KC are staged in two LDS buffers; each thread keeps two slabs of
// global loads in flight.
template <typename T, int TM, int TN, bool COLS = (TM < TN)>
struct Tile {
  // COLS: waves stacked along columns, each holding every row of its
  // columns (needed by the panel-row triangular solve); else along rows
  static constexpr int WR = COLS ? 1 : NW;
  static constexpr int WC = NW / WR;
  static constexpr int WM = TM / WR, WN = TN / WC;
  static constexpr int RB = WM / 16, CB = WN / 16;
  static constexpr int SA = TM + 1;   // transposed A slab stride (odd: conflict-free writes)
  static constexpr int SB = TN + 2;   // B slab stride (keeps pair alignment)
  static constexpr int STAGE = KC * (SA + SB);
  static constexpr int AL = TM * KC / 2 / NT;   // pair loads per thread per slab
  static constexpr int BL = TN * KC / 2 / NT;
  static_assert(AL >= 1 && BL >= 1 && (RB * CB == 8 || RB * CB == 16), "tile shape");
};

// Per-thread global-load descriptors of one k-slab (compile-time counts).
// Every load is issued unconditionally (out-of-range lanes read a valid
// address and discard the value), so the compiler can count the loads in
// flight and the wait before storing a slab covers only that slab's loads:
// the next slab's loads stay in flight behind the MFMA work.  HASW: the
// tile includes the right-hand-side column (w, FP64 storage).
// Round to nearest even FP32 -> BF16 (bit pattern); NaN stays NaN.
__device__ __attribute__((always_inline)) inline short to_bf16(float f) {
  const unsigned u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (short)((u >> 16) | 0x40u);
  return (short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// A slab value as it enters LDS: unchanged (MM = 0), or rounded once to
// BF16 and kept as the FP32 value with those upper 16 bits (MM = 1), so
// that a fragment read takes the upper half without rounding again.
template <int MM, typename T>
__device__ __attribute__((always_inline)) inline T slab_value(T v) {
  if constexpr (MM == 0) {
    return v;
  } else {
    return __uint_as_float((unsigned)(unsigned short)to_bf16(v) << 16);
  }
}

template <typename T, int TM, int TN, bool HASW, bool COLS = (TM < TN), int MM = 0>
struct SlabLoader {
  typedef Tile<T, TM, TN, COLS> TL;
  typedef typename Pair<T>::v P2;
  const T* aptr[TL::AL];
  int ak[TL::AL], arow[TL::AL];
  bool aok[TL::AL];
  const T* bbase[TL::BL];
  const double* bw[TL::BL];
  int bstride[TL::BL], bk[TL::BL], bcol[TL::BL], bn[TL::BL];
  bool isw[TL::BL];
  const int* sperm;
  int K;

  // k runs over [kb, kb + K_): the A operand's columns and the B operand's
  // positions start at kb (folded into the base pointers)
  __device__ __attribute__((always_inline)) inline void init(const Elem<T>& el, int r0, int rlim, int c0, int clim, int K_,
                                                             int kb = 0) {
    const int tid = threadIdx.x;
    sperm = el.sperm + kb;
    K = K_;
#pragma unroll
    for (int q = 0; q < TL::AL; ++q) {
      const int idx = tid + q * NT;
      arow[q] = idx / (KC / 2);
      ak[q] = 2 * (idx % (KC / 2));
      const int row = r0 + arow[q];
      aok[q] = row < rlim;
      aptr[q] = (aok[q] ? el.lrow(row) : el.LU) + kb;
    }
#pragma unroll
    for (int q = 0; q < TL::BL; ++q) {
      const int idx = tid + q * NT;
      bk[q] = idx / (TN / 2);
      bcol[q] = 2 * (idx % (TN / 2));
      const int col = c0 + bcol[q];
      bn[q] = col >= clim ? 0 : (col + 1 >= clim ? 1 : 2);
      isw[q] = false;
      bw[q] = el.A;  // a valid address when unused
      bbase[q] = el.LU;
      bstride[q] = 0;
      if (col < el.n) { bbase[q] = el.LU + col; bstride[q] = el.n; }
      else if (col < el.N) { bbase[q] = el.U12 + (col - el.n); bstride[q] = el.t; }
      else if (HASW && col < clim) { isw[q] = true; bw[q] = el.w; }
    }
  }
  // raw loads only: the values are masked when the slab is stored, two
  // slabs later, so nothing waits for them here
  __device__ __attribute__((always_inline)) inline void load(int ch, P2 (&va)[TL::AL], P2 (&vb)[TL::BL],
                                                             double (&vw)[HASW ? TL::BL : 1]) const {
    const int k0 = ch * KC;
#pragma unroll
    for (int q = 0; q < TL::AL; ++q) {
      const int k = k0 + ak[q];
      va[q] = *reinterpret_cast<const P2*>(aptr[q] + (k < K ? k : 0));
    }
#pragma unroll
    for (int q = 0; q < TL::BL; ++q) {
      const int k = k0 + bk[q];
      const size_t pr = (size_t)sperm[k < K ? k : 0];
      vb[q] = *reinterpret_cast<const P2*>(bbase[q] + pr * bstride[q]);
      if constexpr (HASW) vw[q] = bw[q][isw[q] ? pr : 0];
    }
  }
  __device__ __attribute__((always_inline)) inline void store(int ch, T* stage, const P2 (&va)[TL::AL],
                                                              const P2 (&vb)[TL::BL],
                                                              const double (&vw)[HASW ? TL::BL : 1]) const {
    const int k0 = ch * KC;
    T* As = stage;
    T* Bs = stage + KC * TL::SA;
#pragma unroll
    for (int q = 0; q < TL::AL; ++q) {
      // L enters negated: the accumulators start from the tile's input
      // values, so the MFMA chain computes in - L U directly
      const bool ok = aok[q] && k0 + ak[q] < K;
      As[ak[q] * TL::SA + arow[q]] = ok ? slab_value<MM>(-va[q].x) : T(0);
      As[(ak[q] + 1) * TL::SA + arow[q]] = ok ? slab_value<MM>(-va[q].y) : T(0);
    }
#pragma unroll
    for (int q = 0; q < TL::BL; ++q) {
      const bool ok = k0 + bk[q] < K;
      P2 r;
      r.x = (ok && bn[q] >= 1) ? vb[q].x : T(0);
      r.y = (ok && bn[q] == 2) ? vb[q].y : T(0);
      if constexpr (HASW) {
        if (isw[q]) r.x = ok ? (T)vw[q] : T(0);
      }
      r.x = slab_value<MM>(r.x);
      r.y = slab_value<MM>(r.y);
      *reinterpret_cast<P2*>(Bs + bk[q] * TL::SB + bcol[q]) = r;
    }
  }
};

typedef short bf16x4 __attribute__((ext_vector_type(4)));

// MM = 0: MFMA in T.  MM = 1 (T = float): operands rounded to BF16 (when
// they entered the slab), FP32 accumulation, v_mfma_f32_16x16x16_bf16 (A operand: lane l holds
// A[l % 16][4 (l / 16) + i], B operand: B[4 (l / 16) + i][l % 16], i < 4;
// accumulator as for the FP32 16x16x4 operation).
template <typename T, int TM, int TN, int MM, bool COLS = (TM < TN)>
__device__ __attribute__((always_inline)) inline void slab_mma(const T* stage, int wr0, int wc0,
                                typename Mfma<T>::acc_t (&acc)[Tile<T, TM, TN, COLS>::RB][Tile<T, TM, TN, COLS>::CB]) {
  typedef Tile<T, TM, TN, COLS> TL;
  typedef Mfma<T> MF;
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  if constexpr (MM == 0) {
    const T* As = stage + wr0 + li + lg * TL::SA;
    const T* Bs = stage + KC * TL::SA + wc0 + li + lg * TL::SB;
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      T av[TL::RB], bv[TL::CB];
#pragma unroll
      for (int rb = 0; rb < TL::RB; ++rb) av[rb] = As[4 * ks * TL::SA + 16 * rb];
#pragma unroll
      for (int cb = 0; cb < TL::CB; ++cb) bv[cb] = Bs[4 * ks * TL::SB + 16 * cb];
#pragma unroll
      for (int rb = 0; rb < TL::RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < TL::CB; ++cb) acc[rb][cb] = MF::mac(av[rb], bv[cb], acc[rb][cb]);
    }
  } else {
    static_assert(sizeof(T) == 4 && KC % 16 == 0, "BF16 operands need FP32 slabs");
    const T* As = stage + wr0 + li + 4 * lg * TL::SA;
    const T* Bs = stage + KC * TL::SA + wc0 + li + 4 * lg * TL::SB;
#pragma unroll
    for (int ks = 0; ks < KC / 16; ++ks) {
      bf16x4 av[TL::RB], bv[TL::CB];
#pragma unroll
      for (int rb = 0; rb < TL::RB; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) av[rb][i] = (short)(__float_as_uint(As[(16 * ks + i) * TL::SA + 16 * rb]) >> 16);
#pragma unroll
      for (int cb = 0; cb < TL::CB; ++cb)
#pragma unroll
        for (int i = 0; i < 4; ++i) bv[cb][i] = (short)(__float_as_uint(Bs[(16 * ks + i) * TL::SB + 16 * cb]) >> 16);
#pragma unroll
      for (int rb = 0; rb < TL::RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < TL::CB; ++cb)
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[rb], bv[cb], acc[rb][cb], 0, 0, 0);
    }
  }
}

// acc = in - L[r0:r0+TM, kb:kb+K] * U[kb:kb+K, c0:c0+TN] for the workgroup's
// TM x TN tile (kb = 0 but for the update between the two halves of a
// 128-wide panel); rows >= rlim, cols >= clim and k >= kb+K read as zero.
// The accumulators start from the input values (read while the first slabs
// are in flight) and L enters the MFMAs negated.  Waves are stacked as described for Tile.
// k-slabs of KC go through two LDS stages; each thread keeps
// the global loads of the next two slabs in flight in two register buffers.
// Accumulators initialised with the tile's input values (zero outside
// rlim x clim).  SEG >= 0: every column of the tile lies in that segment, so
// each row is resolved once.
template <typename T, int TM, int TN, int SEG, bool COLS = (TM < TN)>
__device__ __attribute__((always_inline)) inline void tile_inputs(const Elem<T>& el, int r0, int rlim, int c0, int clim,
                                                                  typename Mfma<T>::acc_t (&acc)[Tile<T, TM, TN, COLS>::RB][Tile<T, TM, TN, COLS>::CB]) {
  typedef Tile<T, TM, TN, COLS> TL;
  typedef Mfma<T> MF;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr0 = (wv % TL::WR) * TL::WM, wc0 = (wv / TL::WR) * TL::WN;
#pragma unroll
  for (int rb = 0; rb < TL::RB; ++rb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = r0 + wr0 + 16 * rb + MF::row(lane, v);
      if constexpr (SEG >= 0) {
        const T* ip = el.template in_row<SEG>(row);
        const int base = el.template seg_base<SEG>();
#pragma unroll
        for (int cb = 0; cb < TL::CB; ++cb) {
          const int col = c0 + wc0 + 16 * cb + (lane & 15);
          acc[rb][cb][v] = (row < rlim && col < clim) ? ip[col - base] : T(0);
        }
      } else {
#pragma unroll
        for (int cb = 0; cb < TL::CB; ++cb) {
          const int col = c0 + wc0 + 16 * cb + (lane & 15);
          acc[rb][cb][v] = (row < rlim && col < clim) ? el.in(row, col) : T(0);
        }
      }
    }
}

// Store this wave's accumulators inside rlim x clim; SEG as above.
template <typename T, int TM, int TN, int SEG, bool COLS = (TM < TN)>
__device__ __attribute__((always_inline)) inline void tile_store(const Elem<T>& el, int r0, int rlim, int c0, int clim,
                                                                 typename Mfma<T>::acc_t (&acc)[Tile<T, TM, TN, COLS>::RB][Tile<T, TM, TN, COLS>::CB]) {
  typedef Tile<T, TM, TN, COLS> TL;
  typedef Mfma<T> MF;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr0 = (wv % TL::WR) * TL::WM, wc0 = (wv / TL::WR) * TL::WN;
#pragma unroll
  for (int rb = 0; rb < TL::RB; ++rb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = r0 + wr0 + 16 * rb + MF::row(lane, v);
      if (row < rlim) {
        if constexpr (SEG >= 0) {
          T* op = el.template out_row<SEG>(row);
          const int base = el.template seg_base<SEG>();
#pragma unroll
          for (int cb = 0; cb < TL::CB; ++cb) {
            const int col = c0 + wc0 + 16 * cb + (lane & 15);
            if (col < clim) op[col - base] = acc[rb][cb][v];
          }
        } else {
#pragma unroll
          for (int cb = 0; cb < TL::CB; ++cb) {
            const int col = c0 + wc0 + 16 * cb + (lane & 15);
            if (col < clim) el.st(row, col, acc[rb][cb][v]);
          }
        }
      }
    }
}

// seg: the column segment every column of the tile lies in (0 or 1), or -1
// (uniform across the workgroup, so the branch costs nothing per element)
template <typename T, int TM, int TN, bool COLS = (TM < TN)>
__device__ __attribute__((always_inline)) inline void tile_inputs_seg(const Elem<T>& el, int r0, int rlim, int c0, int clim,
                                                                      typename Mfma<T>::acc_t (&acc)[Tile<T, TM, TN, COLS>::RB][Tile<T, TM, TN, COLS>::CB],
                                                                      int seg) {
  if (seg == 0) tile_inputs<T, TM, TN, 0, COLS>(el, r0, rlim, c0, clim, acc);
  else if (seg == 1) tile_inputs<T, TM, TN, 1, COLS>(el, r0, rlim, c0, clim, acc);
  else tile_inputs<T, TM, TN, -1, COLS>(el, r0, rlim, c0, clim, acc);
}
template <typename T, int TM, int TN, bool COLS = (TM < TN)>
__device__ __attribute__((always_inline)) inline void tile_store_seg(const Elem<T>& el, int r0, int rlim, int c0, int clim,
                                                                     typename Mfma<T>::acc_t (&acc)[Tile<T, TM, TN, COLS>::RB][Tile<T, TM, TN, COLS>::CB],
                                                                     int seg) {
  if (seg == 0) tile_store<T, TM, TN, 0, COLS>(el, r0, rlim, c0, clim, acc);
  else if (seg == 1) tile_store<T, TM, TN, 1, COLS>(el, r0, rlim, c0, clim, acc);
  else tile_store<T, TM, TN, -1, COLS>(el, r0, rlim, c0, clim, acc);
}
// The column segment of tile columns [j0, jl): 0, 1, or -1 when it straddles
// n or holds the right-hand-side column.
__device__ __attribute__((always_inline)) inline int tile_seg(int j0, int jl, int n, int N) {
  return jl <= n ? 0 : (j0 >= n && jl <= N) ? 1 : -1;
}

// The slab loop is unrolled by two so that stage and buffer indices are
// compile-time constants.
template <typename T, int TM, int TN, int MM = 0, bool HASW = false, bool COLS = (TM < TN)>
__device__ __attribute__((always_inline)) inline void gemm_tile(const Elem<T>& el, int r0, int rlim, int c0, int clim, int K, T* smem,
                                 typename Mfma<T>::acc_t (&acc)[Tile<T, TM, TN, COLS>::RB][Tile<T, TM, TN, COLS>::CB],
                                 int seg = -1, int kb = 0) {
  typedef Tile<T, TM, TN, COLS> TL;
  typedef Mfma<T> MF;
  typedef typename Pair<T>::v P2;
  const int wv = threadIdx.x >> 6;
  const int wr0 = (wv % TL::WR) * TL::WM, wc0 = (wv / TL::WR) * TL::WN;
  const int lane = threadIdx.x & 63;
  if (K <= 0) {
    tile_inputs_seg<T, TM, TN, COLS>(el, r0, rlim, c0, clim, acc, seg);
    return;
  }
  const int nch = (K + KC - 1) / KC;
  SlabLoader<T, TM, TN, HASW, COLS, MM> ld;
  ld.init(el, r0, rlim, c0, clim, K, kb);
  T* S0 = smem;
  T* S1 = smem + TL::STAGE;
  P2 a0[TL::AL], b0[TL::BL], a1[TL::AL], b1[TL::BL];
  double w0[HASW ? TL::BL : 1], w1[HASW ? TL::BL : 1];
  // loads past the last slab are issued too (they read valid addresses and
  // are masked): the same loads are in flight on every path, so each wait
  // before a store covers exactly the slab being stored
  ld.load(0, a0, b0, w0);
  ld.load(1, a1, b1, w1);
  // the tile's input values, read while the first slabs are in flight
  tile_inputs_seg<T, TM, TN, COLS>(el, r0, rlim, c0, clim, acc, seg);
  ld.store(0, S0, a0, b0, w0);
  ld.load(2, a0, b0, w0);
  __syncthreads();
  for (int ch = 0; ch < nch; ch += 2) {
    ld.store(ch + 1, S1, a1, b1, w1);
    ld.load(ch + 3, a1, b1, w1);
    slab_mma<T, TM, TN, MM, COLS>(S0, wr0, wc0, acc);
    __syncthreads();
    if (ch + 1 < nch) {
      ld.store(ch + 2, S0, a0, b0, w0);
      ld.load(ch + 4, a0, b0, w0);
      slab_mma<T, TM, TN, MM, COLS>(S1, wr0, wc0, acc);
      __syncthreads();
    }
  }
}

// Visit this wave's accumulator elements as (row, col) of the tile.
template <typename T, int TM, int TN, bool COLS = (TM < TN), typename F = int>
__device__ __attribute__((always_inline)) inline void for_acc(int r0, int c0, typename Mfma<T>::acc_t (&acc)[Tile<T, TM, TN, COLS>::RB][Tile<T, TM, TN, COLS>::CB],
                               F f) {
  typedef Tile<T, TM, TN, COLS> TL;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wr0 = (wv % TL::WR) * TL::WM, wc0 = (wv / TL::WR) * TL::WN;
#pragma unroll
  for (int rb = 0; rb < TL::RB; ++rb)
#pragma unroll
    for (int cb = 0; cb < TL::CB; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        f(r0 + wr0 + 16 * rb + Mfma<T>::row(lane, v), c0 + wc0 + 16 * cb + (lane & 15), acc[rb][cb][v]);
}

// acc element v = f(row, col, value) over this wave's accumulators.
template <typename T, int TM, int TN, bool COLS = (TM < TN), typename F = int>
__device__ __attribute__((always_inline)) inline void map_acc(int r0, int c0, typename Mfma<T>::acc_t (&acc)[Tile<T, TM, TN, COLS>::RB][Tile<T, TM, TN, COLS>::CB],
                               F f) {
  typedef Tile<T, TM, TN, COLS> TL;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wr0 = (wv % TL::WR) * TL::WM, wc0 = (wv / TL::WR) * TL::WN;
#pragma unroll
  for (int rb = 0; rb < TL::RB; ++rb)
#pragma unroll
    for (int cb = 0; cb < TL::CB; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        acc[rb][cb][v] = f(r0 + wr0 + 16 * rb + Mfma<T>::row(lane, v), c0 + wc0 + 16 * cb + (lane & 15), acc[rb][cb][v]);
}

// ---- panel factorisation -------------------------------------------------
// The panel [c0, c1) is factored in sub-panels of SW columns.  Every thread
// owns the same positions for the whole panel: A position p >= c0 belongs
// to thread (p - c0) % NT, slot (p - c0) / NT; C row n + q to thread q % NT,
// slot q / NT.  A sub-panel lives in registers while its columns are
// factored, so a pivot column costs one workgroup barrier and no global
// memory traffic.  Between sub-panels the update is left-looking: the U
// rows above the sub-panel come from the panel's L^{-1} (in LDS), and each
// thread applies the L values of its own rows (re-read from global, written
// there by the same thread's earlier sub-panels).
template <typename T, int QA, int QC, int SW>
struct PanelShape {
  static constexpr int R = QA + QC;
  static constexpr int W = sizeof(T) / 4;  // registers per value
  // L values per row fetched per round trip (keeps x + chunk near 128 regs)
  static constexpr int KCH = (R * 16 * W <= 64) ? 16 : ((R * 8 * W <= 64) ? 8 : 4);
};

struct PanelSmem {
  double cv[2][NW];   // wave maxima, double-buffered by column parity
  int ci[2][NW];      // their positions
};

template <typename T>
struct PanelBufs {
  T* Linv;   // CT x LIS: L_pp^{-1} of the panel's factored columns so far
  T* Xu;     // CT x SWMAX: rows [c0, cs) of the sub-panel (input), then scratch
  T* Ut;     // CT x SWMAX: U rows [c0, cs) of the sub-panel
  T* Lb;     // SWMAX x CT: L(cs:ce, c0:ce) rows of the sub-panel
  T* cand;   // 2 x NW x SWMAX: each wave's best candidate row, by column parity
  T* krow;   // 2 x SWMAX: row at the pivot position before the interchange
  PanelSmem* ps;
};

// Rotate every register row left by one column.
template <typename T, int QA, int QC, int SW>
__device__ __attribute__((always_inline)) inline void rotate_rows(T (&x)[QA][SW], T (&xc)[QC][SW]) {
#pragma unroll
  for (int q = 0; q < QA; ++q) {
    const T f = x[q][0];
#pragma unroll
    for (int j = 0; j + 1 < SW; ++j) x[q][j] = x[q][j + 1];
    x[q][SW - 1] = f;
  }
#pragma unroll
  for (int q = 0; q < QC; ++q) {
    const T f = xc[q][0];
#pragma unroll
    for (int j = 0; j + 1 < SW; ++j) xc[q][j] = xc[q][j + 1];
    xc[q][SW - 1] = f;
  }
}

// A register row moved as 16-byte vectors (the caller guarantees alignment).
template <typename T, int W>
__device__ __attribute__((always_inline)) inline void load_row16(T (&dst)[W], const T* src) {
  const T* s = static_cast<const T*>(__builtin_assume_aligned(src, 16));
#pragma unroll
  for (int j = 0; j < W; ++j) dst[j] = s[j];
}
template <typename T, int W>
__device__ __attribute__((always_inline)) inline void store_row16(T* dst, const T (&src)[W]) {
  T* d = static_cast<T*>(__builtin_assume_aligned(dst, 16));
#pragma unroll
  for (int j = 0; j < W; ++j) d[j] = src[j];
}

template <typename T, int QA, int QC, int SW, int CT>
__device__ __attribute__((always_inline)) void panel_factor(const Elem<T>& el, int* sperm, int c0, int c1,
                                                            const PanelBufs<T>& pb, DeviceStatus* status, int elem) {
  typedef PanelShape<T, QA, QC, SW> PS;
  constexpr int KCH = PS::KCH;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n = el.n, N = el.N;
  // every row of LU and L21 starts on a 16-byte boundary (and so does every
  // sub-panel and chunk below, at multiples of 4 columns): full rows of a
  // sub-panel then move as 16-byte vectors
  const bool vec = (n * sizeof(T)) % 16 == 0 &&
                   ((reinterpret_cast<uintptr_t>(el.LU) | reinterpret_cast<uintptr_t>(el.L21)) & 15) == 0;
  for (int cs = c0; cs < c1; cs += SW) {
    const int sw = min(SW, c1 - cs), kp = cs - c0;
    // the previous sub-panel's stores are read below by other threads (rows
    // change owners through interchanges)
    if (kp > 0) sync_global();
    // (1) the sub-panel columns of every owned row (Crout-updated by the
    //     panel-column GEMM; earlier panels' interchanges via sperm)
    //     (columns < n: LU rows for A positions, L21 rows for C rows)
    T x[QA][SW];
    T xc[QC][SW];
    T* xra[QA];
    T* xrc[QC];
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int p = c0 + tid + NT * q;
      xra[q] = p < n ? el.lrow(p) + cs : nullptr;
    }
#pragma unroll
    for (int q = 0; q < QC; ++q) {
      const int r = n + tid + NT * q;
      xrc[q] = r < N ? el.lrow(r) + cs : nullptr;
    }
    if (sw == SW && vec) {
#pragma unroll
      for (int q = 0; q < QA; ++q) {
        if (xra[q]) {
          load_row16(x[q], xra[q]);
        } else {
#pragma unroll
          for (int j = 0; j < SW; ++j) x[q][j] = T(0);
        }
      }
#pragma unroll
      for (int q = 0; q < QC; ++q) {
        if (xrc[q]) {
          load_row16(xc[q], xrc[q]);
        } else {
#pragma unroll
          for (int j = 0; j < SW; ++j) xc[q][j] = T(0);
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < QA; ++q)
#pragma unroll
        for (int j = 0; j < SW; ++j) x[q][j] = (xra[q] && j < sw) ? xra[q][j] : T(0);
#pragma unroll
      for (int q = 0; q < QC; ++q)
#pragma unroll
        for (int j = 0; j < SW; ++j) xc[q][j] = (xrc[q] && j < sw) ? xrc[q][j] : T(0);
    }
    if (kp > 0) {
      // (2) U rows [c0, cs): Ut = L_pp^{-1}[0:kp, 0:kp] X[c0:cs]; positions
      //     c0 .. cs-1 are slot 0 of threads 0 .. kp-1
      if (tid < kp) {
#pragma unroll
        for (int j = 0; j < SW; ++j) pb.Xu[tid * SW + j] = x[0][j];
      }
      __syncthreads();
      for (int o = tid; o < kp * SW; o += NT) {
        const int i = o / SW, j = o % SW;
        T acc = T(0);
        for (int m = 0; m <= i; ++m) acc += pb.Linv[i * (CT + 1) + m] * pb.Xu[m * SW + j];
        pb.Ut[o] = acc;
      }
      __syncthreads();
      if (tid < kp) {
#pragma unroll
        for (int j = 0; j < SW; ++j) x[0][j] = pb.Ut[tid * SW + j];
      }
      // (3) rows at positions >= cs and the C rows: X -= L[row, c0:cs] Ut,
      //     KCH columns of L per round trip
      const T* lra[QA];
      const T* lrc[QC];
#pragma unroll
      for (int q = 0; q < QA; ++q) {
        const int p = c0 + tid + NT * q;
        lra[q] = (p >= cs && p < n) ? el.lrow(p) + c0 : nullptr;
      }
#pragma unroll
      for (int q = 0; q < QC; ++q) {
        const int r = n + tid + NT * q;
        lrc[q] = r < N ? el.lrow(r) + c0 : nullptr;
      }
      for (int k0 = 0; k0 < kp; k0 += KCH) {
        T la[QA][KCH], lc[QC][KCH];
        if (vec && k0 + KCH <= kp) {
#pragma unroll
          for (int q = 0; q < QA; ++q) {
            if (lra[q]) {
              load_row16(la[q], lra[q] + k0);
            } else {
#pragma unroll
              for (int kk = 0; kk < KCH; ++kk) la[q][kk] = T(0);
            }
          }
#pragma unroll
          for (int q = 0; q < QC; ++q) {
            if (lrc[q]) {
              load_row16(lc[q], lrc[q] + k0);
            } else {
#pragma unroll
              for (int kk = 0; kk < KCH; ++kk) lc[q][kk] = T(0);
            }
          }
        } else {
#pragma unroll
          for (int q = 0; q < QA; ++q)
#pragma unroll
            for (int kk = 0; kk < KCH; ++kk) la[q][kk] = (lra[q] && k0 + kk < kp) ? lra[q][k0 + kk] : T(0);
#pragma unroll
          for (int q = 0; q < QC; ++q)
#pragma unroll
            for (int kk = 0; kk < KCH; ++kk) lc[q][kk] = (lrc[q] && k0 + kk < kp) ? lrc[q][k0 + kk] : T(0);
        }
#pragma unroll
        for (int kk = 0; kk < KCH; ++kk) {
          if (k0 + kk < kp) {
            const T* u = pb.Ut + (k0 + kk) * SW;
#pragma unroll
            for (int j = 0; j < SW; ++j) {
              const T uj = u[j];
#pragma unroll
              for (int q = 0; q < QA; ++q) x[q][j] -= la[q][kk] * uj;
#pragma unroll
              for (int q = 0; q < QC; ++q) xc[q][j] -= lc[q][kk] * uj;
            }
          }
        }
      }
    }
    // (4) partial pivoting, one column at a time, one barrier per column:
    //     each wave posts its best candidate row and the owner of position k
    //     posts row k, so after the barrier every thread can take the pivot
    //     row and perform the interchange.  Buffers alternate by column
    //     parity: a buffer is rewritten only after every wave has passed the
    //     next column's barrier, i.e. finished reading it.
    //     The column loop is not unrolled (it would not fit the instruction
    //     cache): instead every register row is rotated by one after each
    //     column, so the current column always sits in register 0 and
    //     register j holds column kk + j (mod SW).  LDS rows use the same
    //     rotation.
    for (int kk = 0; kk < sw; ++kk) {
      const int k = cs + kk, par = kk & 1;
      T best = T(-1);
      int bq = -1;
#pragma unroll
      for (int q = 0; q < QA; ++q) {
        const int p = c0 + tid + NT * q;
        const T v = fabs(x[q][0]);
        if (p >= k && p < n && v > best) { best = v; bq = q; }
      }
      const int mine = bq >= 0 ? c0 + tid + NT * bq : INT_MAX;
      // the wave's candidate: largest magnitude, ties to the smallest
      // position (best is -1 where a thread has none, never NaN)
      const T wbest = wave_max(best);
      int bidx = wave_min(best == wbest ? mine : INT_MAX);
      // (register rows are named in static branches on the slot, never
      // reached through a pointer to a row, so that they stay in registers;
      // one lane of the wave is active, so one branch runs)
      T* cw = pb.cand + (par * NW + wv) * SW;
      if (mine == bidx && bidx != INT_MAX) {
#pragma unroll
        for (int q = 0; q < QA; ++q)
          if (q == bq) {
#pragma unroll
            for (int j = 0; j < SW; ++j) cw[j] = x[q][j];
          }
      }
      if (lane == 0) { pb.ps->cv[par][wv] = (double)wbest; pb.ps->ci[par][wv] = bidx; }
      const int ko = k - c0;  // owner of position k: thread ko (slot 0, ko < CT <= NT)
      const bool own_k = tid == ko;
      T* kr = pb.krow + par * SW;
      if (own_k) {
#pragma unroll
        for (int j = 0; j < SW; ++j) kr[j] = x[0][j];
      }
      __syncthreads();
      double gbest = pb.ps->cv[par][0];
      bidx = pb.ps->ci[par][0];
      int bw = 0;
#pragma unroll
      for (int i = 1; i < NW; ++i) {
        const double ov = pb.ps->cv[par][i];
        const int oi = pb.ps->ci[par][i];
        // (bitwise operators: no short-circuit branches)
        const bool take = (ov > gbest) | ((ov == gbest) & (oi < bidx));
        gbest = take ? ov : gbest;
        bidx = take ? oi : bidx;
        bw = take ? i : bw;
      }
      int piv = bidx;
      const T* urow = pb.cand + (par * NW + bw) * SW;
      if (piv == INT_MAX || !(gbest > 0.0) || !isfinite(gbest)) {
        if (tid == 0) latch_status(status, IEDG_ERR_SINGULAR, elem);
        piv = k;
        urow = kr;
      }
      T u[SW];
#pragma unroll
      for (int j = 0; j < SW; ++j) u[j] = urow[j];
      const int po = piv - c0;
      const bool own_p = piv != k && tid == po % NT;
      const int sp = po / NT;
      // the interchange (a thread owning both positions holds k in slot 0
      // and the pivot row in a later slot)
      if (own_k) {
#pragma unroll
        for (int j = 0; j < SW; ++j) x[0][j] = u[j];
      }
      if (own_p) {
#pragma unroll
        for (int q = 0; q < QA; ++q)
          if (q == sp) {
#pragma unroll
            for (int j = 0; j < SW; ++j) x[q][j] = kr[j];
          }
      }
      if (tid == 0 && piv != k) {
        const int tmp = sperm[k];
        sperm[k] = sperm[piv];
        sperm[piv] = tmp;
      }
      // eliminate below the pivot: registers 1 .. sw-kk-1 are the columns
      // right of k in this sub-panel (the others hold finished columns)
      // (the pivot row is masked once, so finished columns take l * 0)
      const T rinv = T(1) / u[0];
      const int live = sw - kk;
      T um[SW];
#pragma unroll
      for (int j = 1; j < SW; ++j) um[j] = j < live ? u[j] : T(0);
#pragma unroll
      for (int q = 0; q < QA; ++q) {
        const int p = c0 + tid + NT * q;
        if (p > k && p < n) {
          const T l = x[q][0] * rinv;
          x[q][0] = l;
#pragma unroll
          for (int j = 1; j < SW; ++j) x[q][j] -= l * um[j];
        }
      }
#pragma unroll
      for (int q = 0; q < QC; ++q) {
        if (n + tid + NT * q < N) {
          const T l = xc[q][0] * rinv;
          xc[q][0] = l;
#pragma unroll
          for (int j = 1; j < SW; ++j) xc[q][j] -= l * um[j];
        }
      }
      rotate_rows<T, QA, QC, SW>(x, xc);
    }
    // sw rotations so far; complete a full turn
    for (int r = sw; r < SW; ++r) rotate_rows<T, QA, QC, SW>(x, xc);
    __syncthreads();  // final sperm of this sub-panel
    // (5) write the sub-panel back: U rows above, the factored rows, L below
    //     (row pointers again: interchanges moved rows between positions)
    if (sw == SW && vec) {
#pragma unroll
      for (int q = 0; q < QA; ++q) {
        const int p = c0 + tid + NT * q;
        if (p < n) store_row16(el.lrow(p) + cs, x[q]);
      }
#pragma unroll
      for (int q = 0; q < QC; ++q)
        if (xrc[q]) store_row16(xrc[q], xc[q]);
    } else {
#pragma unroll
      for (int q = 0; q < QA; ++q) {
        const int p = c0 + tid + NT * q;
        if (p < n) {
          T* wr = el.lrow(p) + cs;
#pragma unroll
          for (int j = 0; j < SW; ++j)
            if (j < sw) wr[j] = x[q][j];
        }
      }
#pragma unroll
      for (int q = 0; q < QC; ++q)
        if (xrc[q])
#pragma unroll
          for (int j = 0; j < SW; ++j)
            if (j < sw) xrc[q][j] = xc[q][j];
    }
    // the sub-panel rows' own unit-lower L (positions cs .. cs+sw-1 are
    // slot 0 of threads kp .. kp+sw-1) into Lb[:, kp:kp+sw]
    if (tid >= kp && tid < kp + sw) {
      const int i = tid - kp;
#pragma unroll
      for (int j = 0; j < SW; ++j) pb.Lb[i * CT + kp + j] = (j < i) ? x[0][j] : T(0);
    }
    __syncthreads();
    // their L in the panel's earlier columns: Lb[:, 0:kp] (written by earlier
    // sub-panels, visible since the barrier at the top of this one)
    for (int o = tid; o < sw * kp; o += NT) {
      const int i = o / kp, k = o % kp;
      pb.Lb[i * CT + k] = el.ld(cs + i, c0 + k);
    }
    __syncthreads();
    // (6) grow L_pp^{-1} by rows kp .. kp+sw.  With L = [L11 0; L21 L22]:
    //     inv = [L11^{-1} 0; -L22^{-1} L21 L11^{-1}  L22^{-1}]
    {
      T* Y = pb.Xu;  // sw x kp values, Y[i * CT + k]
      for (int o = tid; o < sw * kp; o += NT) {
        const int i = o / kp, k = o % kp;
        T acc = T(0);
        for (int m = k; m < kp; ++m) acc += pb.Lb[i * CT + m] * pb.Linv[m * (CT + 1) + k];
        Y[i * CT + k] = acc;
      }
      __syncthreads();
      if (tid < sw) {
        const int j = tid;
        for (int i = 0; i < sw; ++i) {
          T acc = (i == j) ? T(1) : T(0);
          if (i > j)
            for (int m = j; m < i; ++m) acc -= pb.Lb[i * CT + kp + m] * pb.Linv[(kp + m) * (CT + 1) + kp + j];
          pb.Linv[(kp + i) * (CT + 1) + kp + j] = acc;
        }
        for (int i = 0; i < j; ++i) pb.Linv[(kp + i) * (CT + 1) + kp + j] = T(0);
      }
      __syncthreads();
      for (int o = tid; o < sw * kp; o += NT) {
        const int i = o / kp, k = o % kp;
        T acc = T(0);
        for (int m = 0; m <= i; ++m) acc += pb.Linv[(kp + i) * (CT + 1) + kp + m] * Y[m * CT + k];
        pb.Linv[(kp + i) * (CT + 1) + k] = -acc;
      }
      __syncthreads();
    }
  }
  sync_global();  // the panel's stores are read by the panel-row GEMM
}

// The right half [cm, c1) of a 128-wide panel whose left half [c0, cm) is
// factored (Linv holds L11^{-1} in its top-left block).  Factoring the two
// halves separately, with one MFMA update between them, replaces the
// left-looking updates of the right half's sub-panels from all 64 left
// columns (each row's L values re-read from global once per sub-panel) by
// one pass over them:
//   (a) U[c0:cm, cm:c1] = L11^{-1} X[c0:cm, cm:c1]   (X staged in LDS)
//   (b) X[cm:N, cm:c1] -= L[cm:N, c0:cm] U[c0:cm, cm:c1]   (256 x 64 tiles,
//       k over [c0, cm); FP32 operands in every operand mode: within a
//       panel the arithmetic stays that of the panel factorisation)
//   (c) the right half by panel_factor, its L22^{-1} in the bottom-right
//       block of Linv (pivoting among positions >= cm moves whole rows,
//       their left-half L values with them)
//   (d) the bottom-left block -L22^{-1} L21 L11^{-1}, with L21 = L[cm:c1,
//       c0:cm] at the final positions.
// sg: the GEMM staging area, free during the panel phase.
template <typename T, int QA, int QC, int SW, int CT>
__device__ __attribute__((always_inline)) void panel_right_half(const Elem<T>& el, int* sperm, int c0, int cm, int c1,
                                                                const PanelBufs<T>& pb, T* sg, DeviceStatus* status,
                                                                int elem) {
  static_assert(CT == 128, "two halves of a 128-wide panel");
  constexpr int H = 64, LS = CT + 1;
  const int tid = threadIdx.x;
  const int wl = cm - c0, wr = c1 - cm;  // wl == H, 0 < wr <= H
  // (a)
  {
    T* X = sg;  // wl x H
    for (int o = tid; o < wl * H; o += NT) {
      const int i = o / H, j = o % H;
      X[o] = j < wr ? el.ld(c0 + i, cm + j) : T(0);
    }
    __syncthreads();
    for (int o = tid; o < wl * H; o += NT) {
      const int i = o / H, j = o % H;
      if (j < wr) {
        T acc = T(0);
        for (int m = 0; m <= i; ++m) acc += pb.Linv[i * LS + m] * X[m * H + j];
        el.lrow(c0 + i)[cm + j] = acc;
      }
    }
    sync_global();
  }
  // (b)
  typedef Tile<T, 256, H> TH;
  for (int r0 = cm; r0 < el.N; r0 += 256) {
    typename Mfma<T>::acc_t acc[TH::RB][TH::CB];
    gemm_tile<T, 256, H, 0>(el, r0, el.N, cm, c1, wl, sg, acc, 0, c0);
    tile_store_seg<T, 256, H>(el, r0, el.N, cm, c1, acc, 0);
  }
  sync_global();
  // (c)
  PanelBufs<T> pr = pb;
  pr.Linv = pb.Linv + wl * LS + wl;
  panel_factor<T, QA, QC, SW, CT>(el, sperm, cm, c1, pr, status, elem);
  // (d) Y = L21 L11^{-1} (L21 staged in LDS), then -L22^{-1} Y
  {
    T* L = sg;          // wr x H
    T* Y = sg + H * H;  // wr x H
    for (int o = tid; o < wr * H; o += NT) {
      const int i = o / H, k = o % H;
      L[o] = el.ld(cm + i, c0 + k);
    }
    __syncthreads();
    for (int o = tid; o < wr * H; o += NT) {
      const int i = o / H, k = o % H;
      T acc = T(0);
      for (int m = k; m < wl; ++m) acc += L[i * H + m] * pb.Linv[m * LS + k];
      Y[o] = acc;
    }
    __syncthreads();
    for (int o = tid; o < wr * H; o += NT) {
      const int i = o / H, k = o % H;
      T acc = T(0);
      for (int m = 0; m <= i; ++m) acc += pb.Linv[(wl + i) * LS + wl + m] * Y[m * H + k];
      pb.Linv[(wl + i) * LS + k] = -acc;
    }
    __syncthreads();
  }
}

// ---- the kernel -------------------------------------------------------------
template <typename T, int CT>
struct CondenseSmem {
  // two stages of the largest tile shape used (elements)
  static constexpr int STAGE_MAX =
      std::max({Tile<T, Shapes<T, CT>::CM, CT>::STAGE, Tile<T, CT, Shapes<T, CT>::RN>::STAGE,
                Tile<T, Shapes<T, CT>::SM, Shapes<T, CT>::SN>::STAGE});
  static constexpr int GEMM = 2 * STAGE_MAX;
  static constexpr int PANEL = CT * (CT + 1) + 2 * CT * SWMAX + SWMAX * CT + 2 * NW * SWMAX + 2 * SWMAX;
  static size_t bytes(int n) {
    return sizeof(T) * (GEMM + PANEL) + sizeof(PanelSmem) + 16 + sizeof(int) * n;
  }
};

// dst[0:len] = (float) src[0:len] by the workgroup; len a multiple of 4,
// 16 values per thread in flight.
__device__ __attribute__((always_inline)) inline void convert_copy(const double* __restrict__ src,
                                                                   float* __restrict__ dst, size_t len) {
  const size_t step = (size_t)NT * 16;
  for (size_t i0 = (size_t)threadIdx.x * 4; i0 < len; i0 += step) {
    double4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const size_t i = i0 + (size_t)u * NT * 4;
      if (i < len) v[u] = *reinterpret_cast<const double4*>(src + i);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const size_t i = i0 + (size_t)u * NT * 4;
      if (i < len) *reinterpret_cast<float4*>(dst + i) = make_float4((float)v[u].x, (float)v[u].y, (float)v[u].z, (float)v[u].w);
    }
  }
}

template <typename T, int QA, int QC, int LW, int MM, int CT>
__device__ __attribute__((always_inline)) void condense_one(const CondenseArgs<T>& a, int e, unsigned char* smem_raw) {
  typedef Mfma<T> MF;
  const int tid = threadIdx.x;
  const int n = a.n, t = a.t, N = n + t;
  T* sg = reinterpret_cast<T*>(smem_raw);
  PanelBufs<T> pb;
  pb.Linv = sg + CondenseSmem<T, CT>::GEMM;
  pb.Xu = pb.Linv + CT * (CT + 1);
  pb.Ut = pb.Xu + CT * SWMAX;
  pb.Lb = pb.Ut + CT * SWMAX;
  pb.cand = pb.Lb + SWMAX * CT;
  pb.krow = pb.cand + 2 * NW * SWMAX;
  pb.ps = reinterpret_cast<PanelSmem*>(pb.krow + 2 * SWMAX);
  int* sperm = reinterpret_cast<int*>(reinterpret_cast<unsigned char*>(pb.ps) + sizeof(PanelSmem) + 16);

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

  for (int i = tid; i < n; i += NT) sperm[i] = i;
  if constexpr (sizeof(T) == 4) {
    convert_copy(el.A, el.LU, nn);
    convert_copy(el.B, el.U12, nt);
    convert_copy(el.C, el.L21, nt);
    convert_copy(el.D, el.Ke, tt);
    sync_global();  // read by other threads below
  } else {
    __syncthreads();
  }

  typedef Shapes<T, CT> SH;
  typedef Tile<T, SH::CM, CT> TA;
  typedef Tile<T, CT, SH::RN> TB;
  typedef Tile<T, SH::SM, SH::SN> TS;
  for (int c0 = 0; c0 < n; c0 += CT) {
    const int c1 = min(c0 + CT, n);
    // 1. panel column in Crout order
    for (int r0 = c0; r0 < N; r0 += SH::CM) {
      typename MF::acc_t acc[TA::RB][TA::CB];
      gemm_tile<T, SH::CM, CT, MM>(el, r0, N, c0, c1, c0, sg, acc, 0);  // columns < c1 <= n
      tile_store_seg<T, SH::CM, CT>(el, r0, N, c0, c1, acc, 0);
    }
    sync_global();
    // 2. factor the panel, growing L_pp^{-1} (a 128-wide panel in two
    //    halves of 64 with one MFMA update between them)
    if constexpr (CT == 128) {
      const int cm = min(c0 + 64, c1);
      panel_factor<T, QA, QC, LW, CT>(el, sperm, c0, cm, pb, a.status, e);
      if (cm < c1) panel_right_half<T, QA, QC, LW, CT>(el, sperm, c0, cm, c1, pb, sg, a.status, e);
    } else {
      panel_factor<T, QA, QC, LW, CT>(el, sperm, c0, c1, pb, a.status, e);
    }
    // the leaves write L_pp^{-1} on and below the diagonal of each 8-row
    // strip only; the triangular solve below reads whole 16 x 16 diagonal
    // blocks, so clear the strictly upper part (and the padding of a
    // narrow last panel)
    const int wp = c1 - c0;
    for (int q = tid; q < CT * CT; q += NT) {
      const int i = q / CT, k = q % CT;
      if (i >= wp || k >= wp || k > i) pb.Linv[i * (CT + 1) + k] = T(0);
    }
    __syncthreads();
    // 3. panel rows with the triangular solve on the accumulators
    for (int j0 = c1; j0 < NC; j0 += SH::RN) {
      const int jl = min(j0 + SH::RN, NC);
      typename MF::acc_t acc[TB::RB][TB::CB];
      const int seg = tile_seg(j0, jl, n, N);
      if (jl > N)  // this tile holds the right-hand-side column
        gemm_tile<T, CT, SH::RN, MM, true>(el, c0, c1, j0, jl, c0, sg, acc);
      else
        gemm_tile<T, CT, SH::RN, MM, false>(el, c0, c1, j0, jl, c0, sg, acc, seg);
      map_acc<T, CT, SH::RN>(c0, j0, acc, [&](int row, int col, T v) __attribute__((always_inline)) -> T {
        return (row < c1 && col < jl) ? v : T(0);
      });
      {
        const int lane = tid & 63, li = lane & 15;
#pragma unroll
        for (int ib = TB::RB - 1; ib >= 0; --ib) {
          typename MF::acc_t nacc[TB::CB];
#pragma unroll
          for (int cb = 0; cb < TB::CB; ++cb) nacc[cb] = MF::zero();
#pragma unroll
          for (int rb = 0; rb <= ib; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const T av = pb.Linv[(16 * ib + li) * (CT + 1) + 16 * rb + MF::row(lane, v)];
#pragma unroll
              for (int cb = 0; cb < TB::CB; ++cb) nacc[cb] = MF::mac(av, acc[rb][cb][v], nacc[cb]);
            }
#pragma unroll
          for (int cb = 0; cb < TB::CB; ++cb) acc[ib][cb] = nacc[cb];
        }
      }
      tile_store_seg<T, CT, SH::RN>(el, c0, c1, j0, jl, acc, seg);
    }
    sync_global();
  }
  // 4. Schur block
  for (int r0 = n; r0 < N; r0 += SH::SM) {
    for (int j0 = n; j0 < NC; j0 += SH::SN) {
      const int jl = min(j0 + SH::SN, NC);
      typename MF::acc_t acc[TS::RB][TS::CB];
      const int seg = tile_seg(j0, jl, n, N);  // 1, or -1 with the right-hand side
      if (jl > N)
        gemm_tile<T, SH::SM, SH::SN, MM, true>(el, r0, N, j0, jl, n, sg, acc);
      else
        gemm_tile<T, SH::SM, SH::SN, MM, false>(el, r0, N, j0, jl, n, sg, acc, seg);
      tile_store_seg<T, SH::SM, SH::SN>(el, r0, N, j0, jl, acc, seg);
    }
  }
  for (int i = tid; i < n; i += NT) a.perm[(size_t)e * n + i] = sperm[i];
  __syncthreads();  // LDS is reused by the next element of a persistent workgroup
}

// One element per workgroup.
template <typename T, int QA, int QC, int LW, int MM, int CT>
__global__ __launch_bounds__(NT) void condense_kernel(CondenseArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  condense_one<T, QA, QC, LW, MM, CT>(a, blockIdx.x, smem_raw);
}

// One item of the batched form, compiled as a function of its own so that
// each size class gets its own register allocation (inlined together, the
// six classes would share, and spill, one allocation).  A callee cannot know
// that its arguments are uniform over the workgroup, so it makes them so
// itself and reads the segment through the constant address space: the
// segment's sizes and pointers then sit in scalar registers as they do in
// the one-element-per-workgroup kernel.
template <typename T, int QA, int QC, int LW, int MM, int CT>
__device__ __noinline__ void condense_item(const CondenseArgs<T>* segs, int seg, int e) {
#if defined(__HIP_DEVICE_COMPILE__)  // address spaces exist only in the device pass
  extern __shared__ __align__(16) unsigned char smem_raw[];
  typedef const __attribute__((address_space(4))) CondenseArgs<T> ConstArgs;
  const uint64_t p = reinterpret_cast<uint64_t>(segs);
  const uint64_t pu = (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)p) |
                      ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(p >> 32)) << 32);
  const CondenseArgs<T> a = ((ConstArgs*)pu)[__builtin_amdgcn_readfirstlane(seg)];
  condense_one<T, QA, QC, LW, MM, CT>(a, __builtin_amdgcn_readfirstlane(e), smem_raw);
#endif
}

// The instantiation of one item's size class, sub-panel width and panel width.
template <typename T, int MM, int CT>
__device__ __forceinline__ void queue_item(const CondenseArgs<T>* segs, int seg, int e, int qa, int qc, int lw) {
  if (qa <= 1 && qc <= 1) {
    if (lw == 16) condense_item<T, 1, 1, 16, MM, CT>(segs, seg, e);
    else condense_item<T, 1, 1, 8, MM, CT>(segs, seg, e);
  } else if (qa <= 3 && qc <= 1) {
    if (lw == 16) condense_item<T, 3, 1, 16, MM, CT>(segs, seg, e);
    else condense_item<T, 3, 1, 8, MM, CT>(segs, seg, e);
  } else {
    if (lw == 16) condense_item<T, 5, 2, 16, MM, CT>(segs, seg, e);
    else condense_item<T, 5, 2, 8, MM, CT>(segs, seg, e);
  }
}

// Batched form, persistent: n_wg workgroups take (segment, element) items
// from a queue (one atomic counter) until it runs dry.  Segments may differ
// in element size: each item runs the instantiation of its size class and of
// its segment's sub-panel and panel widths (a.lw, a.ct), so it computes exactly what the
// one-element-per-workgroup kernel computes for it (bitwise).  The work list
// is ordered largest elements first, so the last items taken are short ones.
template <typename T, int MM>
__global__ __launch_bounds__(NT) void condense_queue_kernel(const CondenseArgs<T>* __restrict__ segs,
                                                            const int2* __restrict__ items, int n_items,
                                                            int* counter) {
  __shared__ int next;
  while (true) {
    if (threadIdx.x == 0) next = atomicAdd(counter, 1);
    __syncthreads();
    // the item index, and so the segment's sizes and pointers, are uniform
    // over the workgroup: keep them in scalar registers
    const int it = __builtin_amdgcn_readfirstlane(next);
    __syncthreads();  // every thread has read `next` before thread 0 overwrites it
    if (it >= n_items) break;
    const int2 w = items[it];
    const int seg = __builtin_amdgcn_readfirstlane(w.x), e = __builtin_amdgcn_readfirstlane(w.y);
    const int n = segs[seg].n, t = segs[seg].t, lw = segs[seg].lw, ct = segs[seg].ct;
    const int qa = (n + NT - 1) / NT, qc = (t + NT - 1) / NT;
    if constexpr (CT_MAX<T> == 128) {
      if (ct == 128) {
        queue_item<T, MM, 128>(segs, seg, e, qa, qc, lw);
        continue;
      }
    }
    queue_item<T, MM, 64>(segs, seg, e, qa, qc, lw);
  }
}

// Resets the queue counter on the stream (a kernel, not a memset, so that the
// pair can be captured in a graph).  A template only so that the precision
// translation units may each instantiate it.
template <typename T>
__global__ void condense_queue_reset_kernel(int* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

template <typename T, int QA, int QC, int LW, int MM, int CT>
hipError_t launch_condense_lw(const CondenseArgs<T>& a, hipStream_t s) {
  const size_t smem = CondenseSmem<T, CT>::bytes(a.n);
  auto kern = condense_kernel<T, QA, QC, LW, MM, CT>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(a.E), dim3(NT), smem, s, a);
  return hipGetLastError();
}

template <typename T, int QA, int QC, int MM, int CT>
hipError_t launch_condense(const CondenseArgs<T>& a, int lw, hipStream_t s) {
  if (lw == 16) return launch_condense_lw<T, QA, QC, 16, MM, CT>(a, s);
  return launch_condense_lw<T, QA, QC, 8, MM, CT>(a, s);
}

template <typename T, int MM, int CT>
hipError_t launch_class(const CondenseArgs<T>& a, int lw, hipStream_t s) {
  const int qa = (a.n + NT - 1) / NT, qc = (a.t + NT - 1) / NT;
  if (qa <= 1 && qc <= 1) return launch_condense<T, 1, 1, MM, CT>(a, lw, s);
  if (qa <= 3 && qc <= 1) return launch_condense<T, 3, 1, MM, CT>(a, lw, s);
  if (qa <= 5 && qc <= 2) return launch_condense<T, 5, 2, MM, CT>(a, lw, s);
  return hipErrorInvalidValue;
}

// Workgroups of the batched form that fit on the device at once (the
// persistent grid) when LDS is sized for n_max local dofs at the widest
// panel.
template <typename T, int MM>
int queue_slots(int n_max) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const size_t smem = CondenseSmem<T, CT_MAX<T>>::bytes(n_max);
  auto kern = condense_queue_kernel<T, MM>;
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)smem) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, NT, smem) != hipSuccess) return 0;
  return cus * per_cu;
}

// The batched form of one precision (and operand mode): every item
// instantiation lives in the persistent kernel, compiled in the translation
// unit of its precision.
template <typename T, int MM>
hipError_t dispatch_queue(hipStream_t s, const CondenseArgs<T>* segs, const int2* items, int n_items, int n_max,
                          int* counter, int n_wg) {
  const size_t smem = CondenseSmem<T, CT_MAX<T>>::bytes(n_max);
  auto kern = condense_queue_kernel<T, MM>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(condense_queue_reset_kernel<T>, dim3(1), dim3(64), 0, s, counter);
  hipLaunchKernelGGL(kern, dim3(n_wg), dim3(NT), smem, s, segs, items, n_items, counter);
  return hipGetLastError();
}

// One launch over elements 0 .. a.E-1 (the one-element-per-workgroup
// kernels of one precision, compiled in a translation unit of their own so
// that the two halves of a precision build in parallel).  lw, ct: sub-panel
// width (8 or 16) and panel width (64 or 128), 0 for the untuned defaults.
template <typename T, int MM>
hipError_t dispatch_single(const CondenseArgs<T>& a, hipStream_t s, int lw, int ct) {
  if (lw == 0) lw = default_leaf_width(sizeof(T), a.n, a.t);
  if (ct == 0) ct = default_panel_width(sizeof(T), a.n);
  if constexpr (CT_MAX<T> == 128) {
    if (ct == 128) return launch_class<T, MM, 128>(a, lw, s);
  }
  return launch_class<T, MM, 64>(a, lw, s);
}

}  // namespace iedg
