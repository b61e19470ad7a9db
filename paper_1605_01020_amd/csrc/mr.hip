// Minimal-residual initial guess for Newton's method (section 2.2.1,
// eq. MinRes2): alpha = argmin over beta of ||R(sum_j beta_j x_j)||^2 over s
// previous solutions x_j = (z_j, uhat_j), by Levenberg-Marquardt with
// finite-difference gradients.  The residual is that of the uncondensed
// Newton system plus a componentwise cubic term:
//   R_NS,e = F_e - A_e z_e - B_e uhat_e - eps z_e^3,
//   R_FL   = G - sum_e P_e^T (C_e z_e + D_e uhat_e) - eps uhat^3.
//
// A residual evaluation is bound by reading the FP64 element blocks (50.8 GB
// at the 16x16x8 p = 3 subdomain), so every pass evaluates a batch of points
// at once: each row of A, B, C, D is read once and dotted with every
// point's (z_e, uhat_e), which are formed in LDS from the previous
// solutions.  Each Levenberg-Marquardt trial is one pass over the blocks:
// the trial point and its s finite-difference neighbours together, so an
// accepted trial already carries the next Jacobian.  The s x s damped
// normal equations are solved on the host from a deterministic Gram matrix
// of the difference vectors and the residual.
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "mesh.h"

namespace iedg {

constexpr int MR_THR = 1024, MR_WAVES = MR_THR / 64;  // 16 waves: enough loads in flight per CU
constexpr int MR_MAXS = 8, MR_MAXM = MR_MAXS + 1;
constexpr int MR_PAIRS = MR_MAXM * (MR_MAXM + 1) / 2;
constexpr int MR_GBLK = 512;  // workgroups of the Gram reduction

// m points, point k = sum_j beta[k][j] x_j.
struct MrPoints {
  int m, s;
  double beta[MR_MAXM][MR_MAXS];
};

// Wave-wide sums of m accumulators (fixed butterfly order).
__device__ __forceinline__ void wave_sum_m(double (&a)[MR_MAXM], int m) {
#pragma unroll
  for (int k = 0; k < MR_MAXM; ++k)
    if (k < m) a[k] = wave_sum(a[k]);
}

// acc[k] += row . vecs[k] (k < m) over len entries, one wave: each lane
// keeps 8 loads of the row in flight; vecs [m][len] in LDS.
__device__ __forceinline__ void row_dots(const double* __restrict__ row, const double* vecs, int len, int m,
                                         double (&acc)[MR_MAXM]) {
  const int lane = threadIdx.x & 63;
  for (int c0 = lane; c0 < len; c0 += 64 * 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = c0 + 64 * u;
      v[u] = c < len ? row[c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = c0 + 64 * u;
      if (c < len) {
#pragma unroll
        for (int k = 0; k < MR_MAXM; ++k)
          if (k < m) acc[k] += v[u] * vecs[(size_t)k * len + c];
      }
    }
  }
}

// One workgroup per element: the points' (z_e, uhat_e) in LDS, then per
// row of [A B] the residual R_NS of every point, per row of [C D] the
// element's contribution q = C z + D uhat of every point, and per point the
// element's sum of R_NS^2.
__global__ __launch_bounds__(MR_THR) void mr_elem_kernel(int n, int t, int b, int S, int E, const int32_t* elem_faces,
                                                         const double* __restrict__ A, const double* __restrict__ B,
                                                         const double* __restrict__ C, const double* __restrict__ D,
                                                         const double* __restrict__ F, const double* __restrict__ Z,
                                                         const double* __restrict__ U, int64_t Nt, double eps,
                                                         MrPoints P, double* R, int64_t L, double* q, double* part) {
  extern __shared__ __align__(16) double msm[];
  const int m = P.m, s = P.s;
  double* zs = msm;                  // [m][n]
  double* us = zs + (size_t)m * n;   // [m][t]
  double* red = us + (size_t)m * t;  // [MR_WAVES][MR_MAXM]
  const int e = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int i = tid; i < n; i += MR_THR) {
    double xj[MR_MAXS];
#pragma unroll
    for (int j = 0; j < MR_MAXS; ++j) xj[j] = j < s ? Z[((size_t)j * E + e) * n + i] : 0.0;
    for (int k = 0; k < m; ++k) {
      double v = 0.0;
#pragma unroll
      for (int j = 0; j < MR_MAXS; ++j)
        if (j < s) v += P.beta[k][j] * xj[j];
      zs[(size_t)k * n + i] = v;
    }
  }
  for (int i = tid; i < t; i += MR_THR) {
    const int a = i / b, l = i - a * b;
    const size_t g = (size_t)elem_faces[S * e + a] * b + l;
    double xj[MR_MAXS];
#pragma unroll
    for (int j = 0; j < MR_MAXS; ++j) xj[j] = j < s ? U[(size_t)j * Nt + g] : 0.0;
    for (int k = 0; k < m; ++k) {
      double v = 0.0;
#pragma unroll
      for (int j = 0; j < MR_MAXS; ++j)
        if (j < s) v += P.beta[k][j] * xj[j];
      us[(size_t)k * t + i] = v;
    }
  }
  __syncthreads();
  const size_t nn = (size_t)n * n, nt = (size_t)n * t, tt = (size_t)t * t;
  double sq[MR_MAXM];
#pragma unroll
  for (int k = 0; k < MR_MAXM; ++k) sq[k] = 0.0;
  // rows of [A B]: R_NS
  for (int i = wv; i < n; i += MR_WAVES) {
    double acc[MR_MAXM];
#pragma unroll
    for (int k = 0; k < MR_MAXM; ++k) acc[k] = 0.0;
    row_dots(A + e * nn + (size_t)i * n, zs, n, m, acc);
    row_dots(B + e * nt + (size_t)i * t, us, t, m, acc);
    wave_sum_m(acc, m);
    if (lane == 0) {
      const double f = F[(size_t)e * n + i];
#pragma unroll
      for (int k = 0; k < MR_MAXM; ++k)
        if (k < m) {
          const double zk = zs[(size_t)k * n + i];
          const double r = f - acc[k] - eps * zk * zk * zk;
          R[(size_t)k * L + (size_t)e * n + i] = r;
          sq[k] += r * r;
        }
    }
  }
  // rows of [C D]: q
  for (int i = wv; i < t; i += MR_WAVES) {
    double acc[MR_MAXM];
#pragma unroll
    for (int k = 0; k < MR_MAXM; ++k) acc[k] = 0.0;
    row_dots(C + e * nt + (size_t)i * n, zs, n, m, acc);
    row_dots(D + e * tt + (size_t)i * t, us, t, m, acc);
    wave_sum_m(acc, m);
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < MR_MAXM; ++k)
        if (k < m) q[((size_t)k * E + e) * t + i] = acc[k];
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < MR_MAXM; ++k) red[wv * MR_MAXM + k] = sq[k];
  }
  __syncthreads();
  if (tid < m) {
    double v = 0.0;
    for (int w = 0; w < MR_WAVES; ++w) v += red[w * MR_MAXM + tid];
    part[(size_t)tid * E + e] = v;
  }
}

// One workgroup (128 threads) per trace unit: R_FL of every point on the
// unit's b dofs (contributions of its element slots in ascending order) and
// the unit's sum of R_FL^2 per point.
__global__ __launch_bounds__(128) void mr_face_kernel(int b, int t, int S, int E, int NF, const int32_t* src_ptr,
                                                      const int32_t* src_list,
                                                      const double* q, const double* G, const double* U, int64_t Nt,
                                                      double eps, MrPoints P, double* R, int64_t L, int64_t En,
                                                      double* part) {
  __shared__ double red[2][MR_MAXM];
  const int f = blockIdx.x, l = threadIdx.x, m = P.m, s = P.s;
  double sq[MR_MAXM];
#pragma unroll
  for (int k = 0; k < MR_MAXM; ++k) sq[k] = 0.0;
  if (l < b) {
    const size_t i = (size_t)f * b + l;
    double xj[MR_MAXS];
#pragma unroll
    for (int j = 0; j < MR_MAXS; ++j) xj[j] = j < s ? U[(size_t)j * Nt + i] : 0.0;
    const double g = G[i];
    const int k0 = src_ptr[f], k1 = src_ptr[f + 1];
#pragma unroll
    for (int k = 0; k < MR_MAXM; ++k) {
      if (k < m) {
        double u = 0.0;
#pragma unroll
        for (int j = 0; j < MR_MAXS; ++j)
          if (j < s) u += P.beta[k][j] * xj[j];
        double v = g;
        for (int c = k0; c < k1; ++c) {
          const int code = src_list[c], e = code / S, a = code - e * S;
          v -= q[((size_t)k * E + e) * t + a * b + l];
        }
        v -= eps * u * u * u;
        R[(size_t)k * L + En + i] = v;
        sq[k] = v * v;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < MR_MAXM; ++k) {
    const double w = wave_sum(sq[k]);
    if ((l & 63) == 0) red[l >> 6][k] = w;
  }
  __syncthreads();
  if (l < m) part[(size_t)l * NF + f] = red[0][l] + red[1][l];
}

// sums[k] = sum of the element partials then the face partials of point k
// (one wave per point, fixed order).
__global__ void mr_sum_kernel(const double* pe, int E, const double* pf, int NF, double* sums) {
  const int k = blockIdx.x, lane = threadIdx.x;
  double v = 0.0;
  for (int i = lane; i < E; i += 64) v += pe[(size_t)k * E + i];
  for (int i = lane; i < NF; i += 64) v += pf[(size_t)k * NF + i];
  v = wave_sum(v);
  if (lane == 0) sums[k] = v;
}

// Difference quotients D_i = (R_i - R_0) / h_i, i = 1 .. s, in place.
__global__ void mr_fd_kernel(double* R, int64_t L, int s, MrPoints H) {
  const int64_t total = (int64_t)s * L;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(x / L) + 1;
    const int64_t j = x - (int64_t)(i - 1) * L;
    R[(size_t)i * L + j] = (R[(size_t)i * L + j] - R[j]) / H.beta[0][i - 1];
  }
}

// Gram matrix of V_a (a < nv): V_a = R_{a+1} for a < nv - 1, V_{nv-1} = R_0.
// Stage 1: MR_GBLK workgroups, each a contiguous chunk, partial products of
// every pair (a <= b, packed) in fixed order; stage 2 sums the chunks.
__global__ __launch_bounds__(256) void mr_gram_part_kernel(const double* R, int64_t L, int nv, double* gpart) {
  __shared__ double red[4][MR_PAIRS];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t chunk = (L + gridDim.x - 1) / gridDim.x;
  const int64_t j0 = (int64_t)blockIdx.x * chunk, j1 = j0 + chunk < L ? j0 + chunk : L;
  double acc[MR_PAIRS];
#pragma unroll
  for (int p = 0; p < MR_PAIRS; ++p) acc[p] = 0.0;
  for (int64_t j = j0 + tid; j < j1; j += 256) {
    double v[MR_MAXM];
#pragma unroll
    for (int a = 0; a < MR_MAXM; ++a) v[a] = a < nv ? R[(size_t)(a + 1 < nv ? a + 1 : 0) * L + j] : 0.0;
    int p = 0;
#pragma unroll
    for (int a = 0; a < MR_MAXM; ++a)
#pragma unroll
      for (int c = a; c < MR_MAXM; ++c, ++p) acc[p] += v[a] * v[c];
  }
#pragma unroll
  for (int p = 0; p < MR_PAIRS; ++p) {
    const double w = wave_sum(acc[p]);
    if (lane == 0) red[wv][p] = w;
  }
  __syncthreads();
  for (int p = tid; p < MR_PAIRS; p += 256) gpart[(size_t)blockIdx.x * MR_PAIRS + p] = red[0][p] + red[1][p] + red[2][p] + red[3][p];
}

__global__ void mr_gram_sum_kernel(const double* gpart, int nblk, double* gram) {
  const int p = blockIdx.x, lane = threadIdx.x;
  double v = 0.0;
  for (int i = lane; i < nblk; i += 64) v += gpart[(size_t)i * MR_PAIRS + p];
  v = wave_sum(v);
  if (lane == 0) gram[p] = v;
}

// z0 = sum_j alpha_j Z_j, u0 = sum_j alpha_j U_j.
__global__ void mr_combine_kernel(const double* Z, int64_t En, const double* U, int64_t Nt, MrPoints P, double* z0,
                                  double* u0) {
  const int64_t total = En + Nt;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    const bool isz = x < En;
    const int64_t i = isz ? x : x - En;
    const double* src = isz ? Z : U;
    const int64_t len = isz ? En : Nt;
    double v = 0.0;
    for (int j = 0; j < P.s; ++j) v += P.beta[0][j] * src[(size_t)j * len + i];
    (isz ? z0 : u0)[i] = v;
  }
}

}  // namespace iedg

using namespace iedg;

struct iedg_mr_s {
  iedg_context ctx = nullptr;
  iedg_mesh mesh = nullptr;
  int n = 0, s_max = 0;
  int64_t L = 0;          // E n + N_t
  double* set[2] = {nullptr, nullptr};  // two sets of (s_max + 1) vectors of L
  double* q = nullptr;    // [(s_max + 1)][E][t]
  double* part = nullptr; // [(s_max + 1)][E + N_f]
  double* sums = nullptr; // [(s_max + 1)]
  double* gpart = nullptr;
  double* gram = nullptr; // [MR_PAIRS]
  double* h_buf = nullptr;  // pinned [MR_PAIRS + MR_MAXM]
};

extern "C" void iedg_mr_destroy(iedg_mr st) {
  if (!st) return;
  for (double* p : {st->set[0], st->set[1], st->q, st->part, st->sums, st->gpart, st->gram})
    if (p) hipFree(p);
  if (st->h_buf) hipHostFree(st->h_buf);
  delete st;
}

extern "C" iedg_status iedg_mr_create(iedg_context ctx, iedg_mesh mesh, int32_t n_local, int32_t s_max, iedg_mr* out) {
  if (!ctx || !mesh || !out || n_local <= 0) return set_error(ctx, IEDG_ERR_INVALID_ARG, "mr_create: bad arguments");
  if (s_max < 1 || s_max > MR_MAXS)
    return set_error(ctx, IEDG_ERR_UNSUPPORTED, "mr_create: s_max=%d (1 .. %d)", s_max, MR_MAXS);
  *out = nullptr;
  auto* st = new iedg_mr_s();
  st->ctx = ctx;
  st->mesh = mesh;
  st->n = n_local;
  st->s_max = s_max;
  st->L = (int64_t)mesh->n_elem * n_local + mesh->n_trace;
  const size_t nv = (size_t)s_max + 1;
  hipError_t e = hipSuccess;
  for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipMalloc(&st->set[k], sizeof(double) * nv * st->L);
  if (e == hipSuccess) e = hipMalloc(&st->q, sizeof(double) * nv * mesh->n_elem * mesh->t);
  if (e == hipSuccess) e = hipMalloc(&st->part, sizeof(double) * nv * (mesh->n_elem + mesh->n_face));
  if (e == hipSuccess) e = hipMalloc(&st->sums, sizeof(double) * nv);
  if (e == hipSuccess) e = hipMalloc(&st->gpart, sizeof(double) * MR_GBLK * MR_PAIRS);
  if (e == hipSuccess) e = hipMalloc(&st->gram, sizeof(double) * MR_PAIRS);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&st->h_buf), sizeof(double) * (MR_PAIRS + MR_MAXM),
                                         hipHostMallocDefault);
  if (e != hipSuccess) {
    iedg_mr_destroy(st);
    return set_error(ctx, e == hipErrorOutOfMemory ? IEDG_ERR_OOM : IEDG_ERR_HIP, "mr_create: %s",
                     hipGetErrorString(e));
  }
  *out = st;
  return IEDG_OK;
}

namespace {

struct MrInputs {
  const double *A, *B, *C, *D, *F, *G, *Z, *U;
  double eps;
  int s;
};

// R[k] (k < P.m) = R(point k) into R [m][L], sums[k] = ||R[k]||^2.
iedg_status mr_pass(iedg_mr st, const MrInputs& in, const MrPoints& P, double* R, double* sums, hipStream_t stream) {
  iedg_context ctx = st->ctx;
  iedg_mesh mesh = st->mesh;
  const int n = st->n, t = mesh->t, b = mesh->b, E = mesh->n_elem, NF = mesh->n_face;
  const size_t smem = sizeof(double) * ((size_t)P.m * (n + t) + MR_WAVES * MR_MAXM);
  if (smem > 160 * 1024)
    return set_error(ctx, IEDG_ERR_UNSUPPORTED, "mr: %d points of n=%d t=%d exceed LDS", P.m, n, t);
  IEDG_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void*>(mr_elem_kernel),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
  double* pe = st->part;
  double* pf = st->part + (size_t)P.m * E;
  hipLaunchKernelGGL(mr_elem_kernel, dim3(E), dim3(MR_THR), smem, stream, n, t, b, mesh->slots, E, mesh->d_elem_faces, in.A, in.B,
                     in.C, in.D, in.F, in.Z, in.U, (int64_t)mesh->n_trace, in.eps, P, R, st->L, st->q, pe);
  hipLaunchKernelGGL(mr_face_kernel, dim3(NF), dim3(128), 0, stream, b, t, mesh->slots, E, NF, mesh->d_src_ptr,
                     mesh->d_src_list, st->q, in.G, in.U,
                     (int64_t)mesh->n_trace, in.eps, P, R, st->L, (int64_t)E * n, pf);
  hipLaunchKernelGGL(mr_sum_kernel, dim3(P.m), dim3(64), 0, stream, pe, E, pf, NF, sums);
  IEDG_LAUNCH_CHECK(ctx, "mr pass launch");
  return IEDG_OK;
}

// The trial point beta and its s forward-difference neighbours (steps h).
MrPoints fd_points(const std::vector<double>& beta, double fd, std::vector<double>& h) {
  MrPoints P{};
  const int s = (int)beta.size();
  P.m = s + 1;
  P.s = s;
  h.assign(s, 0.0);
  for (int k = 0; k <= s; ++k)
    for (int j = 0; j < s; ++j) P.beta[k][j] = beta[j];
  for (int i = 0; i < s; ++i) {
    h[i] = fd * std::max(1.0, std::fabs(beta[i]));
    P.beta[i + 1][i] += h[i];
  }
  return P;
}

// Solve M d = r (s x s, row-major) by Gaussian elimination with partial
// pivoting; false if a pivot is zero or not finite.
bool small_solve(std::vector<double> M, std::vector<double> r, int s, std::vector<double>& d) {
  for (int k = 0; k < s; ++k) {
    int p = k;
    for (int i = k + 1; i < s; ++i)
      if (std::fabs(M[i * s + k]) > std::fabs(M[p * s + k])) p = i;
    if (!(std::fabs(M[p * s + k]) > 0.0) || !std::isfinite(M[p * s + k])) return false;
    if (p != k) {
      for (int j = 0; j < s; ++j) std::swap(M[k * s + j], M[p * s + j]);
      std::swap(r[k], r[p]);
    }
    for (int i = k + 1; i < s; ++i) {
      const double f = M[i * s + k] / M[k * s + k];
      for (int j = k; j < s; ++j) M[i * s + j] -= f * M[k * s + j];
      r[i] -= f * r[k];
    }
  }
  d.assign(s, 0.0);
  for (int k = s - 1; k >= 0; --k) {
    double v = r[k];
    for (int j = k + 1; j < s; ++j) v -= M[k * s + j] * d[j];
    d[k] = v / M[k * s + k];
  }
  for (double v : d)
    if (!std::isfinite(v)) return false;
  return true;
}

}  // namespace

extern "C" iedg_status iedg_mr_residual(iedg_context ctx, iedg_mr st, const double* A, const double* B,
                                        const double* C, const double* D, const double* F, const double* G,
                                        double eps, int32_t s, const double* Zprev, const double* Uprev, int32_t m,
                                        const double* beta, double* R, double* sums, hipStream_t stream) {
  if (!ctx || !st || !A || !B || !C || !D || !F || !G || !Zprev || !Uprev || !beta || !R || !sums)
    return set_error(ctx, IEDG_ERR_INVALID_ARG, "mr_residual: null argument");
  if (s < 1 || s > st->s_max || m < 1 || m > st->s_max + 1)
    return set_error(ctx, IEDG_ERR_INVALID_ARG, "mr_residual: s=%d m=%d (s_max %d)", s, m, st->s_max);
  MrPoints P{};
  P.m = m;
  P.s = s;
  for (int k = 0; k < m; ++k)
    for (int j = 0; j < s; ++j) P.beta[k][j] = beta[(size_t)k * s + j];
  return mr_pass(st, MrInputs{A, B, C, D, F, G, Zprev, Uprev, eps, s}, P, R, sums, stream);
}

extern "C" iedg_status iedg_mr_guess(iedg_context ctx, iedg_mr st, const double* A, const double* B, const double* C,
                                     const double* D, const double* F, const double* G, double eps, int32_t s,
                                     const double* Zprev, const double* Uprev, const iedg_mr_opts* opts,
                                     double* alpha, double* z0, double* u0, iedg_mr_info* info, hipStream_t stream) {
  if (!ctx || !st || !A || !B || !C || !D || !F || !G || !Zprev || !Uprev || !alpha || !z0 || !u0)
    return set_error(ctx, IEDG_ERR_INVALID_ARG, "mr_guess: null argument");
  if (s < 1 || s > st->s_max) return set_error(ctx, IEDG_ERR_INVALID_ARG, "mr_guess: s=%d (s_max %d)", s, st->s_max);
  const int max_iters = opts ? opts->max_iters : 20;
  const double lambda0 = opts ? opts->lambda0 : 1e-3, fd = opts ? opts->fd_step : 1e-7, tol = opts ? opts->tol : 1e-10;
  const double ftol = opts ? opts->ftol : 1e-10;
  if (max_iters < 0 || !(lambda0 > 0.0) || !(fd > 0.0) || !(tol >= 0.0) || !(ftol >= 0.0))
    return set_error(ctx, IEDG_ERR_INVALID_ARG, "mr_guess: bad options");
  const MrInputs in{A, B, C, D, F, G, Zprev, Uprev, eps, s};
  const int nv = s + 1;
  const int64_t L = st->L;
  double* h = st->h_buf;
  int cur = 0, passes = 0;
  auto read = [&](const double* src, int count) -> iedg_status {
    IEDG_HIP(ctx, hipMemcpyAsync(h, src, sizeof(double) * count, hipMemcpyDeviceToHost, stream));
    IEDG_HIP(ctx, hipStreamSynchronize(stream));
    return IEDG_OK;
  };
  // H = J^T J and g = J^T r of the set holding the accepted point: the
  // columns of J become difference quotients in place, then the Gram matrix
  // of (J columns, r) is read back
  std::vector<double> Hm(s * s), g(s), hstep;
  auto jacobian = [&](int set, const std::vector<double>& hs) -> iedg_status {
    MrPoints Hp{};
    for (int i = 0; i < s; ++i) Hp.beta[0][i] = hs[i];
    hipLaunchKernelGGL(mr_fd_kernel, dim3(1024), dim3(256), 0, stream, st->set[set], L, s, Hp);
    hipLaunchKernelGGL(mr_gram_part_kernel, dim3(MR_GBLK), dim3(256), 0, stream, st->set[set], L, nv, st->gpart);
    hipLaunchKernelGGL(mr_gram_sum_kernel, dim3(MR_PAIRS), dim3(64), 0, stream, st->gpart, MR_GBLK, st->gram);
    IEDG_LAUNCH_CHECK(ctx, "mr jacobian launch");
    iedg_status e = read(st->gram, MR_PAIRS);
    if (e != IEDG_OK) return e;
    // packed pairs (a <= c) over MR_MAXM slots: a, c < nv map to the same
    // packed index as in the kernel
    auto pk = [&](int a, int c) {
      int p = 0;
      for (int x = 0; x < a; ++x) p += MR_MAXM - x;
      return p + (c - a);
    };
    for (int i = 0; i < s; ++i) {
      for (int j = 0; j < s; ++j) Hm[i * s + j] = h[pk(std::min(i, j), std::max(i, j))];
      g[i] = h[pk(i, nv - 1)];
    }
    return IEDG_OK;
  };
  std::vector<double> beta(s, 0.0), hs;
  beta[0] = 1.0;
  MrPoints P = fd_points(beta, fd, hs);
  iedg_status e = mr_pass(st, in, P, st->set[cur], st->sums, stream);
  if (e != IEDG_OK) return e;
  ++passes;
  if ((e = read(st->sums, 1)) != IEDG_OK) return e;
  double obj = h[0];
  const double obj0 = obj;
  double lam = lambda0;
  int iters = 0;
  if (obj > 0.0 && max_iters > 0) {
    if ((e = jacobian(cur, hs)) != IEDG_OK) return e;
  }
  while (iters < max_iters && obj > 0.0) {
    bool accepted = false;
    double decrease = 0.0;
    std::vector<double> d;
    for (int tries = 0; tries < 10; ++tries) {
      std::vector<double> Md(Hm), rhs(s);
      for (int i = 0; i < s; ++i) {
        Md[i * s + i] += lam * Hm[i * s + i];
        rhs[i] = -g[i];
      }
      if (!small_solve(Md, rhs, s, d)) break;
      std::vector<double> bt(s), ht;
      for (int i = 0; i < s; ++i) bt[i] = beta[i] + d[i];
      MrPoints Pt = fd_points(bt, fd, ht);
      if ((e = mr_pass(st, in, Pt, st->set[1 - cur], st->sums, stream)) != IEDG_OK) return e;
      ++passes;
      if ((e = read(st->sums, 1)) != IEDG_OK) return e;
      const double ot = h[0];
      if (ot < obj) {
        decrease = obj - ot;
        cur = 1 - cur;
        beta = bt;
        hs = ht;
        obj = ot;
        lam = std::max(lam / 10.0, 1e-12);
        accepted = true;
        break;
      }
      lam *= 10.0;
    }
    if (!accepted) break;
    ++iters;
    double dmax = 0.0, bmax = 0.0;
    for (int i = 0; i < s; ++i) {
      dmax = std::max(dmax, std::fabs(d[i]));
      bmax = std::max(bmax, std::fabs(beta[i]));
    }
    if (dmax <= tol * (1.0 + bmax) || decrease <= ftol * (obj + decrease) || !(obj > 0.0) || iters >= max_iters)
      break;
    if ((e = jacobian(cur, hs)) != IEDG_OK) return e;
  }
  MrPoints Pa{};
  Pa.m = 1;
  Pa.s = s;
  for (int j = 0; j < s; ++j) {
    Pa.beta[0][j] = beta[j];
    alpha[j] = beta[j];
  }
  const int64_t En = (int64_t)st->mesh->n_elem * st->n;
  hipLaunchKernelGGL(mr_combine_kernel, dim3(1024), dim3(256), 0, stream, Zprev, En, Uprev,
                     (int64_t)st->mesh->n_trace, Pa, z0, u0);
  IEDG_LAUNCH_CHECK(ctx, "mr combine launch");
  if (info) {
    info->iters = iters;
    info->passes = passes;
    info->obj0 = obj0;
    info->obj = obj;
  }
  return IEDG_OK;
}
