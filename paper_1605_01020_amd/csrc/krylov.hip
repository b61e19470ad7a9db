// Restarted GMRES(m), left preconditioned by BILU(0), with classical
// Gram-Schmidt applied twice per Arnoldi step (section 2.2.2, eq. LS1;
// Saad and Schultz 1986).  Every Krylov quantity is FP64.  Reductions are
// two-stage with a fixed chunk-to-workgroup map, so results are bitwise
// reproducible.
#include <cmath>

#include "common.h"
#include "mesh.h"

namespace iedg {

iedg_status spmv_launch(iedg_context ctx, iedg_mesh m, iedg_prec kprec, const void* K, const double* x,
                        const double* rhs, double* y, int mode, hipStream_t stream, const int* skip);
iedg_status ilu0_apply_launch(iedg_context ctx, iedg_mesh m, iedg_prec mprec, const void* M, const double* x,
                              double* y, hipStream_t stream, const int* skip);
iedg_status ras_apply_launch(iedg_context ctx, iedg_ras ras, iedg_prec mprec, const void* Mloc, const double* x,
                             double* y, hipStream_t stream, const int* skip);

constexpr int KTHR = 256;
constexpr int KPER = 8;                 // values per thread per chunk
constexpr int KCH = KTHR * KPER;        // chunk length per workgroup
constexpr int MAXV = 256;               // max Krylov vectors per cycle + 2

// partial[c * ld + k] = sum over chunk c of V_k . w   (k < nv), and, when
// self >= 0, partial[c * ld + self] = w . w
__global__ __launch_bounds__(KTHR) void dots_kernel(const double* V, int64_t ldv, int nv, const double* w,
                                                    int64_t N, double* partial, int ld, int self, const int* skip) {
  __shared__ double red[KTHR / 64];
  if (skip && *skip) return;
  const int c = blockIdx.x;
  const int64_t base = (int64_t)c * KCH;
  double wv[KPER];
#pragma unroll
  for (int q = 0; q < KPER; ++q) {
    const int64_t i = base + threadIdx.x + (int64_t)q * KTHR;
    wv[q] = i < N ? w[i] : 0.0;
  }
  for (int k = 0; k < nv; ++k) {
    const double* v = V + (int64_t)k * ldv;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < KPER; ++q) {
      const int64_t i = base + threadIdx.x + (int64_t)q * KTHR;
      if (i < N) s += v[i] * wv[q];
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) partial[(int64_t)c * ld + k] = s;
  }
  if (self >= 0) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < KPER; ++q) s += wv[q] * wv[q];
    s = block_sum(s, red);
    if (threadIdx.x == 0) partial[(int64_t)c * ld + self] = s;
  }
}

// Each workgroup reduces partial_in (nb chunks, fixed order) to h[0:nv],
// then w[chunk] -= sum_k h_k V_k[chunk].  Workgroup 0 stores h into
// hcol (accumulate = 0: overwrite, 1: add).  Afterwards, when next_dots,
// partial_out[c][k] = V_k . w over the chunk (k < nv); otherwise
// partial_out[c][0] = w . w over the chunk.
__global__ __launch_bounds__(KTHR) void cgs_update_kernel(const double* V, int64_t ldv, int nv, double* w,
                                                          int64_t N, const double* partial_in, int nb, int ld_in,
                                                          double* hcol, int accumulate, double* partial_out,
                                                          int ld_out, int next_dots, const int* skip) {
  __shared__ double h[MAXV];
  __shared__ double red[KTHR / 64];
  if (skip && *skip) return;
  const int c = blockIdx.x;
  for (int k = threadIdx.x; k < nv; k += KTHR) {
    double s = 0.0;
    for (int q = 0; q < nb; ++q) s += partial_in[(int64_t)q * ld_in + k];
    h[k] = s;
  }
  __syncthreads();
  if (c == 0)
    for (int k = threadIdx.x; k < nv; k += KTHR) hcol[k] = accumulate ? hcol[k] + h[k] : h[k];
  const int64_t base = (int64_t)c * KCH;
  double wv[KPER];
#pragma unroll
  for (int q = 0; q < KPER; ++q) {
    const int64_t i = base + threadIdx.x + (int64_t)q * KTHR;
    wv[q] = i < N ? w[i] : 0.0;
  }
  for (int k = 0; k < nv; ++k) {
    const double* v = V + (int64_t)k * ldv;
    const double hk = h[k];
#pragma unroll
    for (int q = 0; q < KPER; ++q) {
      const int64_t i = base + threadIdx.x + (int64_t)q * KTHR;
      if (i < N) wv[q] -= hk * v[i];
    }
  }
#pragma unroll
  for (int q = 0; q < KPER; ++q) {
    const int64_t i = base + threadIdx.x + (int64_t)q * KTHR;
    if (i < N) w[i] = wv[q];
  }
  if (next_dots) {
    for (int k = 0; k < nv; ++k) {
      const double* v = V + (int64_t)k * ldv;
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < KPER; ++q) {
        const int64_t i = base + threadIdx.x + (int64_t)q * KTHR;
        if (i < N) s += v[i] * wv[q];
      }
      s = block_sum(s, red);
      if (threadIdx.x == 0) partial_out[(int64_t)c * ld_out + k] = s;
    }
  } else {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < KPER; ++q) s += wv[q] * wv[q];
    s = block_sum(s, red);
    if (threadIdx.x == 0) partial_out[(int64_t)c * ld_out] = s;
  }
}

// Scalars shared between the Arnoldi kernels and the host readback.
struct GmresScal {
  double est;       // |g_{j+1}|
  double hn;        // ||w|| after orthogonalisation
  double wn0;       // ||w|| before orthogonalisation
  double inv_scale; // 1 / value used by scale_kernel
  double norm;      // a norm requested by the host
  double nR;        // ||R|| (device-driven cycle)
  double inner_tol; // inner stopping threshold (device-driven cycle)
  double rho;       // true relative residual at the end of the cycle
  int done;         // inner loop finished: later Arnoldi kernels return at once
  int k;            // Arnoldi steps taken in the cycle
  int converged;
  int pad;
};

// Reduce nb partial sums -> sqrt, fixed order (one thread).
__device__ inline double reduce_sqrt(const double* partial, int nb, int ld, int idx) {
  double s = 0.0;
  for (int q = 0; q < nb; ++q) s += partial[(int64_t)q * ld + idx];
  return sqrt(s);
}

// Finish Arnoldi step j: H[j+1, j] = ||w||, apply the stored rotations to
// column j, form the new rotation and update g.  One thread.
__global__ void arnoldi_finish_kernel(const double* partial_norm, int nb, const double* partial_w0, int ld_w0,
                                      int idx_w0, double* H, int ldh, int j, double* cs, double* sn, double* g,
                                      GmresScal* sc, int device_control, int steps) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (device_control && sc->done) return;
  const double hn = reduce_sqrt(partial_norm, nb, 1, 0);
  const double wn0 = reduce_sqrt(partial_w0, nb, ld_w0, idx_w0);
  double* hc = H + (int64_t)j * ldh;
  hc[j + 1] = hn;
  for (int i = 0; i < j; ++i) {
    const double a = hc[i], b = hc[i + 1];
    hc[i] = cs[i] * a + sn[i] * b;
    hc[i + 1] = -sn[i] * a + cs[i] * b;
  }
  const double a = hc[j], b = hc[j + 1];
  double c = 1.0, s = 0.0, r = a;
  if (b != 0.0) {
    r = hypot(a, b);
    c = a / r;
    s = b / r;
  }
  cs[j] = c;
  sn[j] = s;
  hc[j] = r;
  hc[j + 1] = 0.0;
  const double gj = g[j];
  g[j + 1] = -s * gj;
  g[j] = c * gj;
  sc->est = fabs(g[j + 1]);
  sc->hn = hn;
  sc->wn0 = wn0;
  sc->inv_scale = hn > 0.0 ? 1.0 / hn : 0.0;
  if (device_control) {
    sc->k = j + 1;
    if (!(sc->est > sc->inner_tol) || hn <= 1e-14 * wn0 || j + 1 >= steps) sc->done = 1;
  }
}

// sc->norm = sqrt(sum of partials); sc->inv_scale = 1 / norm; optionally g = (norm, 0, ...)
__global__ void norm_finish_kernel(const double* partial, int nb, int ld, int idx, GmresScal* sc, double* g,
                                   int m1) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double nrm = reduce_sqrt(partial, nb, ld, idx);
  sc->norm = nrm;
  sc->inv_scale = nrm > 0.0 ? 1.0 / nrm : 0.0;
  if (g) {
    g[0] = nrm;
    for (int i = 1; i < m1; ++i) g[i] = 0.0;
  }
}

__global__ void scale_kernel(double* v, int64_t N, const GmresScal* sc, const int* skip) {
  if (skip && *skip) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) v[i] *= sc->inv_scale;
}

// dst = src * inv_scale (device-driven cycle: v0 = M^{-1} R / ||M^{-1} R||)
__global__ void scale_copy_kernel(double* dst, const double* src, int64_t N, const GmresScal* sc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) dst[i] = src[i] * sc->inv_scale;
}

// Device-driven cycle bookkeeping after a norm was reduced into sc->norm.
//   mode 0: norm = ||R||          -> nR, reset flags (done when R = 0)
//   mode 1: norm = ||M^{-1} R||   -> inner threshold
//   mode 2: norm = ||R - K x||    -> rho, converged
__global__ void gmres_dev_set_kernel(GmresScal* sc, int mode, double rtol, double inner_factor) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (mode == 0) {
    sc->nR = sc->norm;
    sc->k = 0;
    sc->converged = 0;
    sc->done = sc->norm == 0.0 ? 1 : 0;
    sc->rho = 0.0;
  } else if (mode == 1) {
    sc->inner_tol = inner_factor * rtol * sc->norm;
  } else {
    sc->rho = sc->nR > 0.0 ? sc->norm / sc->nR : 0.0;
    sc->converged = sc->rho <= rtol ? 1 : 0;
  }
}

__global__ void fill_kernel(double* v, int64_t N, double val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) v[i] = val;
}

__global__ void copy_kernel(double* dst, const double* src, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) dst[i] = src[i];
}

// Back substitution H(0:k, 0:k) y = g(0:k), upper triangular.  One thread.
// When sc is given, k is the device-side step count.
__global__ void hsolve_kernel(const double* H, int ldh, const double* g, int k, double* y, const GmresScal* sc) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (sc) k = sc->k;
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int j = i + 1; j < k; ++j) s -= H[(int64_t)j * ldh + i] * y[j];
    y[i] = s / H[(int64_t)i * ldh + i];
  }
}

// x += sum_{k < nv} y_k V_k
__global__ void multi_axpy_kernel(double* x, const double* V, int64_t ldv, int nv, const double* y, int64_t N,
                                  const GmresScal* sc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  if (sc) nv = sc->k;
  double s = x[i];
  for (int k = 0; k < nv; ++k) s += y[k] * V[(int64_t)k * ldv + i];
  x[i] = s;
}

__global__ void axpy_kernel(int64_t n, double alpha, const double* x, double* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += alpha * x[i];
}

static inline unsigned grid1(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace iedg

using namespace iedg;

extern "C" iedg_status iedg_axpy(iedg_context ctx, int64_t n, double alpha, const double* x, double* y,
                                 hipStream_t stream) {
  if (!ctx || n < 0 || (n > 0 && (!x || !y))) return IEDG_ERR_INVALID_ARG;
  if (n == 0) return IEDG_OK;
  hipLaunchKernelGGL(axpy_kernel, dim3(grid1(n)), dim3(256), 0, stream, n, alpha, x, y);
  IEDG_LAUNCH_CHECK(ctx, "axpy launch");
  return IEDG_OK;
}

// ---- GMRES workspace (the state) ----------------------------------------------
// Everything a solve needs beyond its inputs and outputs is allocated when
// the state is created: the Krylov basis, reduction partials, Hessenberg
// matrix, rotations, the device scalars, pinned host slots for reading them
// back and two events.  Solves and enqueues only launch kernels and copy.
struct iedg_gmres_state_s {
  iedg_mesh mesh = nullptr;
  int steps = 0, nb = 0, ldp = 0;
  int64_t N = 0, ldv = 0;
  double* buf = nullptr;
  double *V, *tmp, *P1, *P2, *P3, *H, *CS, *SN, *G, *Y;
  GmresScal* SC;
  GmresScal* h_sc = nullptr;   // pinned: [0] cycle-end readback, [1..2] chunk flags
  hipEvent_t ev[2] = {nullptr, nullptr};
  iedg_ras ras = nullptr;      // preconditioner: RAS when set, else BILU(0) of the mesh
};

// M^{-1} x with the state's preconditioner.
static iedg_status apply_precond(iedg_context ctx, iedg_mesh mesh, iedg_gmres_state st, iedg_prec mprec,
                                 const void* M, const double* x, double* y, hipStream_t stream, const int* skip) {
  if (st->ras) return ras_apply_launch(ctx, st->ras, mprec, M, x, y, stream, skip);
  return ilu0_apply_launch(ctx, mesh, mprec, M, x, y, stream, skip);
}

extern "C" iedg_status iedg_gmres_state_set_ras(iedg_context ctx, iedg_gmres_state st, iedg_ras ras) {
  if (!ctx || !st) return IEDG_ERR_INVALID_ARG;
  if (ras && ras_mesh(ras) != st->mesh)
    return set_error(ctx, IEDG_ERR_INVALID_ARG, "gmres_state_set_ras: the RAS belongs to another mesh");
  st->ras = ras;
  return IEDG_OK;
}

extern "C" void iedg_gmres_state_destroy(iedg_gmres_state st) {
  if (!st) return;
  if (st->buf) hipFree(st->buf);
  if (st->h_sc) hipHostFree(st->h_sc);
  for (hipEvent_t e : st->ev)
    if (e) hipEventDestroy(e);
  delete st;
}

extern "C" iedg_status iedg_gmres_state_create(iedg_context ctx, iedg_mesh mesh, int32_t steps,
                                               iedg_gmres_state* out) {
  if (!ctx || !mesh || !out || steps < 1 || steps > MAXV - 2)
    return set_error(ctx, IEDG_ERR_INVALID_ARG, "gmres_state_create: steps %d outside [1, %d]", steps, MAXV - 2);
  auto* st = new iedg_gmres_state_s();
  st->mesh = mesh;
  st->steps = steps;
  st->N = mesh->n_trace;
  st->nb = (int)((st->N + KCH - 1) / KCH);
  st->ldp = steps + 2;
  st->ldv = (st->N + 63) & ~int64_t(63);
  size_t off = 0;
  auto take = [&](size_t count) { size_t o = off; off += (count + 63) & ~size_t(63); return o; };
  const int m = steps;
  const size_t oV = take((size_t)(m + 1) * st->ldv), oT = take(st->ldv), oP1 = take((size_t)st->nb * st->ldp),
               oP2 = take((size_t)st->nb * st->ldp), oP3 = take((size_t)st->nb), oH = take((size_t)(m + 1) * m),
               oCS = take(m), oSN = take(m), oG = take(m + 1), oY = take(m), oSC = take(sizeof(GmresScal) / 8 + 1);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&st->buf), off * sizeof(double));
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&st->h_sc), 3 * sizeof(GmresScal), hipHostMallocDefault);
  for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&st->ev[i], hipEventDisableTiming);
  if (e != hipSuccess) {
    iedg_gmres_state_destroy(st);
    return set_error(ctx, IEDG_ERR_OOM, "gmres_state_create: %zu bytes: %s", off * sizeof(double),
                     hipGetErrorString(e));
  }
  double* W = st->buf;
  st->V = W + oV; st->tmp = W + oT; st->P1 = W + oP1; st->P2 = W + oP2; st->P3 = W + oP3; st->H = W + oH;
  st->CS = W + oCS; st->SN = W + oSN; st->G = W + oG; st->Y = W + oY;
  st->SC = reinterpret_cast<GmresScal*>(W + oSC);
  *out = st;
  return IEDG_OK;
}

// Arnoldi steps the host enqueues between two looks at the device's stop
// flag (the look at a chunk happens while the next chunk is already queued).
constexpr int GMRES_CHUNK = 4;

// Arnoldi step j of a cycle under device control (sc->done set by the
// stopping rule makes every later kernel of the cycle return at once).
static iedg_status arnoldi_step(iedg_context ctx, iedg_mesh mesh, iedg_gmres_state st, iedg_prec kprec,
                                const void* Kbsr, iedg_prec mprec, const void* Mbsr, int precond, int j, int steps,
                                hipStream_t stream) {
  const int64_t N = st->N, ldv = st->ldv;
  const int nb = st->nb, ldp = st->ldp, ldh = st->steps + 1;
  const int* done = &st->SC->done;
  double* vj = st->V + (int64_t)j * ldv;
  double* w = st->V + (int64_t)(j + 1) * ldv;
  iedg_status s;
  if ((s = spmv_launch(ctx, mesh, kprec, Kbsr, vj, nullptr, st->tmp, 0, stream, done)) != IEDG_OK) return s;
  if (precond) {
    if ((s = apply_precond(ctx, mesh, st, mprec, Mbsr, st->tmp, w, stream, done)) != IEDG_OK) return s;
  } else {
    hipLaunchKernelGGL(copy_kernel, dim3(grid1(N)), dim3(256), 0, stream, w, st->tmp, N);
  }
  const int nv = j + 1;
  double* hcol = st->H + (int64_t)j * ldh;
  // pass 1 dots (+ ||w||^2 before orthogonalisation at index nv)
  hipLaunchKernelGGL(dots_kernel, dim3(nb), dim3(KTHR), 0, stream, st->V, ldv, nv, w, N, st->P1, ldp, nv, done);
  // pass 1 update + pass 2 dots
  hipLaunchKernelGGL(cgs_update_kernel, dim3(nb), dim3(KTHR), 0, stream, st->V, ldv, nv, w, N, st->P1, nb, ldp,
                     hcol, 0, st->P2, ldp, 1, done);
  // pass 2 update + ||w||^2
  hipLaunchKernelGGL(cgs_update_kernel, dim3(nb), dim3(KTHR), 0, stream, st->V, ldv, nv, w, N, st->P2, nb, ldp,
                     hcol, 1, st->P3, 1, 0, done);
  hipLaunchKernelGGL(arnoldi_finish_kernel, dim3(1), dim3(64), 0, stream, st->P3, nb, st->P1, ldp, nv, st->H, ldh,
                     j, st->CS, st->SN, st->G, st->SC, 1, steps);
  hipLaunchKernelGGL(scale_kernel, dim3(grid1(N)), dim3(256), 0, stream, w, N, st->SC, done);
  IEDG_LAUNCH_CHECK(ctx, "arnoldi launch");
  return IEDG_OK;
}

__global__ void gmres_cycle_begin_kernel(GmresScal* sc) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  sc->done = 0;
  sc->k = 0;
}

extern "C" iedg_status iedg_gmres_solve(iedg_context ctx, iedg_mesh mesh, iedg_gmres_state st, iedg_prec kprec,
                                        const void* Kbsr, iedg_prec mprec, const void* Mbsr, const double* R,
                                        double* x, const iedg_gmres_opts* opts, iedg_gmres_info* info,
                                        hipStream_t stream) {
  if (!ctx || !mesh || !st || !Kbsr || !R || !x || !opts) return set_error(ctx, IEDG_ERR_INVALID_ARG, "gmres: null argument");
  if (st->mesh != mesh) return set_error(ctx, IEDG_ERR_INVALID_ARG, "gmres: the state belongs to another mesh");
  const int m = opts->restart;
  if (m < 1 || m > st->steps)
    return set_error(ctx, IEDG_ERR_INVALID_ARG, "gmres: restart %d outside [1, %d] (the state's size)", m, st->steps);
  if (opts->precond && !Mbsr) return set_error(ctx, IEDG_ERR_INVALID_ARG, "gmres: precond without factors");
  if (!(opts->rtol > 0.0)) return set_error(ctx, IEDG_ERR_INVALID_ARG, "gmres: rtol must be > 0");
  if (opts->max_iters < 0) return set_error(ctx, IEDG_ERR_INVALID_ARG, "gmres: max_iters < 0");
  const int64_t N = st->N, ldv = st->ldv;
  const int nb = st->nb, ldh = st->steps + 1;
  GmresScal* SC = st->SC;
  double *V = st->V, *tmp = st->tmp, *P3 = st->P3;
  auto precond = [&](const double* in, double* out) -> iedg_status {
    if (opts->precond) return apply_precond(ctx, mesh, st, mprec, Mbsr, in, out, stream, nullptr);
    hipLaunchKernelGGL(copy_kernel, dim3(grid1(N)), dim3(256), 0, stream, out, in, N);
    return IEDG_OK;
  };
  auto vnorm = [&](const double* v, double* ginit) {
    hipLaunchKernelGGL(dots_kernel, dim3(nb), dim3(KTHR), 0, stream, v, ldv, 0, v, N, P3, 1, 0, nullptr);
    hipLaunchKernelGGL(norm_finish_kernel, dim3(1), dim3(64), 0, stream, P3, nb, 1, 0, SC, ginit, ldh);
  };
  iedg_status s;
  // x0 = 0; ||R|| and the inner threshold inner_factor * rtol * ||M^{-1} R||, on the device
  hipLaunchKernelGGL(fill_kernel, dim3(grid1(N)), dim3(256), 0, stream, x, N, 0.0);
  vnorm(R, nullptr);
  hipLaunchKernelGGL(gmres_dev_set_kernel, dim3(1), dim3(64), 0, stream, SC, 0, opts->rtol, opts->inner_factor);
  if ((s = precond(R, tmp)) != IEDG_OK) return s;
  vnorm(tmp, nullptr);
  hipLaunchKernelGGL(gmres_dev_set_kernel, dim3(1), dim3(64), 0, stream, SC, 1, opts->rtol, opts->inner_factor);
  iedg_gmres_info inf{0, 0, 0, 0.0};
  GmresScal* hsc = st->h_sc;
  bool first = true;
  while (true) {
    // true residual r = R - K x (x = 0 on the first cycle) and rho = ||r|| / ||R||
    if (first) {
      hipLaunchKernelGGL(copy_kernel, dim3(grid1(N)), dim3(256), 0, stream, tmp, R, N);
    } else {
      if ((s = spmv_launch(ctx, mesh, kprec, Kbsr, x, R, tmp, 1, stream, nullptr)) != IEDG_OK) return s;
    }
    vnorm(tmp, nullptr);
    hipLaunchKernelGGL(gmres_dev_set_kernel, dim3(1), dim3(64), 0, stream, SC, 2, opts->rtol, opts->inner_factor);
    IEDG_LAUNCH_CHECK(ctx, "gmres cycle launch");
    // the cycle-end readback: the only point where the host waits for the stream
    IEDG_HIP(ctx, hipMemcpyAsync(&hsc[0], SC, sizeof(GmresScal), hipMemcpyDeviceToHost, stream));
    IEDG_HIP(ctx, hipStreamSynchronize(stream));
    if (first) {
      if (!std::isfinite(hsc[0].nR)) return set_error(ctx, IEDG_ERR_NONFINITE, "gmres: right-hand side is not finite");
      if (hsc[0].nR == 0.0) { inf.converged = 1; break; }
    } else {
      inf.iters += hsc[0].k;
    }
    const double rho = hsc[0].rho;
    inf.rel_resid = rho;
    if (!std::isfinite(rho)) return set_error(ctx, IEDG_ERR_NONFINITE, "gmres: residual is not finite");
    if (hsc[0].converged) { inf.converged = 1; break; }
    if (inf.iters >= opts->max_iters) break;
    first = false;
    inf.cycles++;
    // v0 = M^{-1} r / ||M^{-1} r||,  g = (beta, 0, ...)
    hipLaunchKernelGGL(gmres_cycle_begin_kernel, dim3(1), dim3(64), 0, stream, SC);
    if ((s = precond(tmp, V)) != IEDG_OK) return s;
    vnorm(V, st->G);
    hipLaunchKernelGGL(scale_kernel, dim3(grid1(N)), dim3(256), 0, stream, V, N, SC, nullptr);
    const int steps = std::min(m, opts->max_iters - inf.iters);
    // Arnoldi steps in chunks: after queueing chunk c the host reads the stop
    // flag that chunk c-1 left (its copy was queued behind it), so the device
    // never waits for the host; steps queued after the stop return at once
    int j = 0, c = 0;
    bool stop = false;
    while (j < steps && !stop) {
      const int j1 = std::min(steps, j + GMRES_CHUNK);
      for (; j < j1; ++j)
        if ((s = arnoldi_step(ctx, mesh, st, kprec, Kbsr, mprec, Mbsr, opts->precond, j, steps, stream)) != IEDG_OK)
          return s;
      IEDG_HIP(ctx, hipMemcpyAsync(&hsc[1 + (c & 1)], SC, sizeof(GmresScal), hipMemcpyDeviceToHost, stream));
      IEDG_HIP(ctx, hipEventRecord(st->ev[c & 1], stream));
      if (c > 0) {
        IEDG_HIP(ctx, hipEventSynchronize(st->ev[(c - 1) & 1]));
        stop = hsc[1 + ((c - 1) & 1)].done != 0;
      }
      ++c;
    }
    hipLaunchKernelGGL(hsolve_kernel, dim3(1), dim3(64), 0, stream, st->H, ldh, st->G, 0, st->Y, SC);
    hipLaunchKernelGGL(multi_axpy_kernel, dim3(grid1(N)), dim3(256), 0, stream, x, V, ldv, 0, st->Y, N, SC);
    IEDG_LAUNCH_CHECK(ctx, "gmres update launch");
  }
  if (info) *info = inf;
  if (!inf.converged)
    return set_error(ctx, IEDG_ERR_NOT_CONVERGED, "gmres: %d iterations, relative residual %.3e > %.3e", inf.iters,
                     inf.rel_resid, opts->rtol);
  return IEDG_OK;
}

// ---- capturable GMRES cycle ------------------------------------------------
extern "C" iedg_status iedg_gmres_enqueue(iedg_context ctx, iedg_mesh mesh, iedg_gmres_state st, iedg_prec kprec,
                                          const void* Kbsr, iedg_prec mprec, const void* Mbsr, const double* R,
                                          double* x, double rtol, double inner_factor, hipStream_t stream) {
  if (!ctx || !mesh || !st || st->mesh != mesh || !Kbsr || !Mbsr || !R || !x || !(rtol > 0.0))
    return set_error(ctx, IEDG_ERR_INVALID_ARG, "gmres_enqueue: bad arguments");
  const int64_t N = st->N, ldv = st->ldv;
  const int nb = st->nb, ldp = st->ldp, m = st->steps;
  double *V = st->V, *tmp = st->tmp, *P1 = st->P1, *P2 = st->P2, *P3 = st->P3, *H = st->H;
  GmresScal* SC = st->SC;
  const int* done = &SC->done;
  iedg_status s;
  hipLaunchKernelGGL(fill_kernel, dim3(grid1(N)), dim3(256), 0, stream, x, N, 0.0);
  // ||R||
  hipLaunchKernelGGL(dots_kernel, dim3(nb), dim3(KTHR), 0, stream, R, ldv, 0, R, N, P3, 1, 0, nullptr);
  hipLaunchKernelGGL(norm_finish_kernel, dim3(1), dim3(64), 0, stream, P3, nb, 1, 0, SC, nullptr, m + 1);
  hipLaunchKernelGGL(gmres_dev_set_kernel, dim3(1), dim3(64), 0, stream, SC, 0, rtol, inner_factor);
  // v0 = M^{-1} R / ||M^{-1} R||, g = (beta, 0, ...)
  if ((s = apply_precond(ctx, mesh, st, mprec, Mbsr, R, tmp, stream, done)) != IEDG_OK) return s;
  hipLaunchKernelGGL(dots_kernel, dim3(nb), dim3(KTHR), 0, stream, tmp, ldv, 0, tmp, N, P3, 1, 0, done);
  hipLaunchKernelGGL(norm_finish_kernel, dim3(1), dim3(64), 0, stream, P3, nb, 1, 0, SC, st->G, m + 1);
  hipLaunchKernelGGL(gmres_dev_set_kernel, dim3(1), dim3(64), 0, stream, SC, 1, rtol, inner_factor);
  hipLaunchKernelGGL(scale_copy_kernel, dim3(grid1(N)), dim3(256), 0, stream, V, tmp, N, SC);
  for (int j = 0; j < m; ++j) {
    double* vj = V + (int64_t)j * ldv;
    double* w = V + (int64_t)(j + 1) * ldv;
    if ((s = spmv_launch(ctx, mesh, kprec, Kbsr, vj, nullptr, tmp, 0, stream, done)) != IEDG_OK) return s;
    if ((s = apply_precond(ctx, mesh, st, mprec, Mbsr, tmp, w, stream, done)) != IEDG_OK) return s;
    const int nv = j + 1;
    double* hcol = H + (int64_t)j * (m + 1);
    hipLaunchKernelGGL(dots_kernel, dim3(nb), dim3(KTHR), 0, stream, V, ldv, nv, w, N, P1, ldp, nv, done);
    hipLaunchKernelGGL(cgs_update_kernel, dim3(nb), dim3(KTHR), 0, stream, V, ldv, nv, w, N, P1, nb, ldp, hcol, 0, P2,
                       ldp, 1, done);
    hipLaunchKernelGGL(cgs_update_kernel, dim3(nb), dim3(KTHR), 0, stream, V, ldv, nv, w, N, P2, nb, ldp, hcol, 1, P3,
                       1, 0, done);
    hipLaunchKernelGGL(arnoldi_finish_kernel, dim3(1), dim3(64), 0, stream, P3, nb, P1, ldp, nv, H, m + 1, j, st->CS,
                       st->SN, st->G, SC, 1, m);
    hipLaunchKernelGGL(scale_kernel, dim3(grid1(N)), dim3(256), 0, stream, w, N, SC, done);
  }
  hipLaunchKernelGGL(hsolve_kernel, dim3(1), dim3(64), 0, stream, H, m + 1, st->G, 0, st->Y, SC);
  hipLaunchKernelGGL(multi_axpy_kernel, dim3(grid1(N)), dim3(256), 0, stream, x, V, ldv, 0, st->Y, N, SC);
  // true residual
  if ((s = spmv_launch(ctx, mesh, kprec, Kbsr, x, R, tmp, 1, stream, nullptr)) != IEDG_OK) return s;
  hipLaunchKernelGGL(dots_kernel, dim3(nb), dim3(KTHR), 0, stream, tmp, ldv, 0, tmp, N, P3, 1, 0, nullptr);
  hipLaunchKernelGGL(norm_finish_kernel, dim3(1), dim3(64), 0, stream, P3, nb, 1, 0, SC, nullptr, m + 1);
  hipLaunchKernelGGL(gmres_dev_set_kernel, dim3(1), dim3(64), 0, stream, SC, 2, rtol, inner_factor);
  IEDG_LAUNCH_CHECK(ctx, "gmres_enqueue launch");
  return IEDG_OK;
}

extern "C" iedg_status iedg_gmres_state_read(iedg_context ctx, iedg_gmres_state st, iedg_gmres_info* info) {
  if (!ctx || !st || !info) return IEDG_ERR_INVALID_ARG;
  GmresScal h;
  IEDG_HIP(ctx, hipMemcpy(&h, st->SC, sizeof(h), hipMemcpyDeviceToHost));
  info->iters = h.k;
  info->cycles = 1;
  info->converged = h.converged;
  info->rel_resid = h.rho;
  return IEDG_OK;
}
