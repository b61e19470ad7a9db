// Element-local kernels on gfx950: recovery of the element unknowns
// (section 2.2.1) and the FP64 residual of the uncondensed Newton system.
#include <mutex>

#include "common.h"
#include "mesh.h"

namespace iedg {

constexpr int LTHR = 256;
constexpr int LWAVES = LTHR / 64;

// z_e = U^{-1} (w_e - U12_e uhat_e): one workgroup per element.  Position i
// of the factorisation lives in physical row perm[i] of LU, U12 and w.
// Rows are processed four per wave at a time (wave_dot_rows) so each lane
// keeps 16 loads in flight; 64-row diagonal blocks of U are staged in LDS in
// the storage precision and solved by one wave.  LDS stays small so that
// several elements share a CU.
template <typename T>
__global__ __launch_bounds__(LTHR) void backsolve_kernel(int n, int t, int b, int S, const int32_t* elem_faces, const T* LU,
                                                         const int32_t* perm, const T* U12, const double* w,
                                                         const double* uhat, double* z) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* ue = reinterpret_cast<double*>(smem_raw);  // t
  double* y = ue + t;                                // n
  int* sp = reinterpret_cast<int*>(y + n);           // n
  T* blk = reinterpret_cast<T*>(sp + ((n + 3) & ~3));  // 64 x 65
  const int e = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int i = tid; i < t; i += LTHR) {
    const int a = i / b, l = i % b;
    ue[i] = uhat[(size_t)elem_faces[S * e + a] * b + l];
  }
  for (int i = tid; i < n; i += LTHR) sp[i] = perm[(size_t)e * n + i];
  __syncthreads();
  const T* U12e = U12 + (size_t)e * n * t;
  for (int i = 4 * wv; i < n; i += 4 * LWAVES) {
    const T* rows[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) rows[r] = U12e + (size_t)sp[min(i + r, n - 1)] * t;
    double s[4];
    wave_dot_rows<T, 4>(rows, ue, t, s);
    if (lane < 4 && i + lane < n) {
      double v = s[0];
#pragma unroll
      for (int r = 1; r < 4; ++r) v = lane == r ? s[r] : v;
      y[i + lane] = w[(size_t)e * n + sp[i + lane]] - v;
    }
  }
  __syncthreads();
  const T* U = LU + (size_t)e * n * n;
  const int nblk = (n + 63) / 64;
  for (int bi = nblk - 1; bi >= 0; --bi) {
    const int i0 = bi * 64, i1 = min(i0 + 64, n), bw = i1 - i0;
    // y[i0:i1] -= U[i0:i1, i1:n] z[i1:n]   (z stored in y beyond i1)
    if (i1 < n) {
      for (int i = i0 + 4 * wv; i < i1; i += 4 * LWAVES) {
        const T* rows[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) rows[r] = U + (size_t)sp[min(i + r, i1 - 1)] * n + i1;
        double s[4];
        wave_dot_rows<T, 4>(rows, y + i1, n - i1, s);
        if (lane < 4 && i + lane < i1) {
          double v = s[0];
#pragma unroll
          for (int r = 1; r < 4; ++r) v = lane == r ? s[r] : v;
          y[i + lane] -= v;
        }
      }
    }
    for (int q = tid; q < 64 * 64; q += LTHR) {
      const int rr = q / 64, cc = q % 64;
      blk[rr * 65 + cc] = (rr < bw && cc < bw && cc >= rr) ? U[(size_t)sp[i0 + rr] * n + i0 + cc] : T(0);
    }
    __syncthreads();
    if (wv == 0) {
      double yl = lane < bw ? y[i0 + lane] : 0.0;
      for (int k = bw - 1; k >= 0; --k) {
        const double zk = __shfl(yl, k, kWave) / (double)blk[k * 65 + k];
        if (lane == k) yl = zk;
        if (lane < k) yl -= (double)blk[lane * 65 + k] * zk;
      }
      if (lane < bw) y[i0 + lane] = yl;
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += LTHR) z[(size_t)e * n + i] = y[i];
}

// Per element: rF_e = F_e - A_e z_e - B_e u_e; q_e = C_e z_e + D_e u_e; also
// per-element sums of rF^2 and F^2 (fixed-order block reduction).
__global__ __launch_bounds__(LTHR) void residual_elem_kernel(int n, int t, int b, int S, const int32_t* elem_faces,
                                                             const double* A, const double* B, const double* C,
                                                             const double* D, const double* F, const double* z,
                                                             const double* uhat, double* rF, double* q,
                                                             double* part_rf, double* part_f) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* ue = reinterpret_cast<double*>(smem_raw);  // t
  double* ze = ue + t;                               // n
  double* red = ze + n;                              // LWAVES
  double* acc = red + LWAVES;                        // 2 * LWAVES
  const int e = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int i = tid; i < t; i += LTHR) {
    const int a = i / b, l = i % b;
    ue[i] = uhat[(size_t)elem_faces[S * e + a] * b + l];
  }
  for (int i = tid; i < n; i += LTHR) ze[i] = z[(size_t)e * n + i];
  __syncthreads();
  const size_t nn = (size_t)n * n, nt = (size_t)n * t, tt = (size_t)t * t;
  const double *Ae = A + e * nn, *Be = B + e * nt, *Ce = C + e * nt, *De = D + e * tt;
  double srf = 0.0, sf = 0.0;  // per-wave partials (lane 0)
  for (int i = wv; i < n; i += LWAVES) {
    const double s = wave_dot<double>(Ae + (size_t)i * n, ze, n) + wave_dot<double>(Be + (size_t)i * t, ue, t);
    if (lane == 0) {
      const double f = F[(size_t)e * n + i];
      const double v = f - s;
      rF[(size_t)e * n + i] = v;
      srf += v * v;
      sf += f * f;
    }
  }
  for (int i = wv; i < t; i += LWAVES) {
    const double s = wave_dot<double>(Ce + (size_t)i * n, ze, n) + wave_dot<double>(De + (size_t)i * t, ue, t);
    if (lane == 0) q[(size_t)e * t + i] = s;
  }
  if (lane == 0) { acc[2 * wv] = srf; acc[2 * wv + 1] = sf; }
  __syncthreads();
  if (tid == 0) {
    double a0 = 0.0, a1 = 0.0;
    for (int k = 0; k < LWAVES; ++k) { a0 += acc[2 * k]; a1 += acc[2 * k + 1]; }
    part_rf[e] = a0;
    part_f[e] = a1;
  }
}

// rG = G - sum_e P_e^T q_e (list order: ascending e, a) and per-unit sums of
// rG^2, G^2 (b <= 128 dofs a unit, one workgroup of 128 threads a unit).
__global__ __launch_bounds__(128) void residual_face_kernel(int b, int t, int S, const int32_t* src_ptr,
                                                            const int32_t* src_list, const double* q,
                                                            const double* G, double* rG, double* part_rg,
                                                            double* part_g) {
  __shared__ double red[2];
  const int f = blockIdx.x, l = threadIdx.x;
  double v = 0.0, g = 0.0;
  if (l < b) {
    const size_t i = (size_t)f * b + l;
    g = G[i];
    v = g;
    for (int k = src_ptr[f]; k < src_ptr[f + 1]; ++k) {
      const int code = src_list[k], e = code / S, a = code - e * S;
      v -= q[(size_t)e * t + a * b + l];
    }
    rG[i] = v;
  }
  const double s1 = wave_sum(l < 64 ? v * v : 0.0) + 0.0;
  const double s2 = wave_sum(l < 64 ? g * g : 0.0);
  const double s3 = wave_sum(l >= 64 ? v * v : 0.0);
  const double s4 = wave_sum(l >= 64 ? g * g : 0.0);
  if (l == 64) { red[0] = s3; red[1] = s4; }
  __syncthreads();
  if (l == 0) {
    part_rg[f] = s1 + red[0];
    part_g[f] = s2 + red[1];
  }
}

// sums[k] = sum over i < len_k of part_k[i], fixed order, one wave each.
__global__ void sum4_kernel(const double* p0, int64_t n0, const double* p1, int64_t n1, const double* p2, int64_t n2,
                            const double* p3, int64_t n3, double* sums) {
  const int k = blockIdx.x, lane = threadIdx.x;
  const double* p = k == 0 ? p0 : k == 1 ? p1 : k == 2 ? p2 : p3;
  const int64_t n = k == 0 ? n0 : k == 1 ? n1 : k == 2 ? n2 : n3;
  double s = 0.0;
  for (int64_t i = lane; i < n; i += 64) s += p[i];
  s = wave_sum(s);
  if (lane == 0) sums[k] = s;
}

}  // namespace iedg

using namespace iedg;

extern "C" iedg_status iedg_backsolve_local(iedg_context ctx, iedg_mesh mesh, int32_t n_local, iedg_prec prec,
                                            const void* LU, const int32_t* perm, const void* U12, const double* w,
                                            const double* uhat, double* z, hipStream_t stream) {
  if (!ctx || !mesh || !LU || !perm || !U12 || !w || !uhat || !z || n_local <= 0) return IEDG_ERR_INVALID_ARG;
  const int n = n_local, t = mesh->t, b = mesh->b;
  const size_t smem_ints = sizeof(double) * (t + n) + sizeof(int) * ((n + 3) & ~3);
  if (prec == IEDG_F64) {
    const size_t smem = smem_ints + sizeof(double) * 64 * 65;
    auto k = backsolve_kernel<double>;
    IEDG_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
    hipLaunchKernelGGL(k, dim3(mesh->n_elem), dim3(LTHR), smem, stream, n, t, b, mesh->slots, mesh->d_elem_faces,
                       (const double*)LU, perm, (const double*)U12, w, uhat, z);
  } else {
    const size_t smem = smem_ints + sizeof(float) * 64 * 65;
    auto k = backsolve_kernel<float>;
    IEDG_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
    hipLaunchKernelGGL(k, dim3(mesh->n_elem), dim3(LTHR), smem, stream, n, t, b, mesh->slots, mesh->d_elem_faces,
                       (const float*)LU, perm, (const float*)U12, w, uhat, z);
  }
  IEDG_LAUNCH_CHECK(ctx, "backsolve launch");
  return IEDG_OK;
}

namespace iedg {

// Both residual entry points: `work` holds q [E][t] and the partial sums
// (2E + 2 n_face values); every entry is written before it is read.
static iedg_status residual_launch(iedg_context ctx, iedg_mesh mesh, int n, const double* A, const double* B,
                                   const double* C, const double* D, const double* F, const double* G,
                                   const double* z, const double* uhat, double* rF, double* rG, double* sums,
                                   double* work, hipStream_t stream) {
  const int t = mesh->t, b = mesh->b, E = mesh->n_elem, NF = mesh->n_face;
  double* q = work;
  double* prf = q + (size_t)E * t;
  double* pf = prf + E;
  double* prg = pf + E;
  double* pg = prg + NF;
  const size_t smem = sizeof(double) * (t + n + 3 * LWAVES);
  IEDG_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void*>(residual_elem_kernel),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
  hipLaunchKernelGGL(residual_elem_kernel, dim3(E), dim3(LTHR), smem, stream, n, t, b, mesh->slots, mesh->d_elem_faces, A, B, C, D,
                     F, z, uhat, rF, q, prf, pf);
  hipLaunchKernelGGL(residual_face_kernel, dim3(NF), dim3(128), 0, stream, b, t, mesh->slots, mesh->d_src_ptr,
                     mesh->d_src_list, q, G, rG, prg, pg);
  hipLaunchKernelGGL(sum4_kernel, dim3(4), dim3(64), 0, stream, prf, (int64_t)E, prg, (int64_t)NF, pf, (int64_t)E, pg,
                     (int64_t)NF, sums);
  IEDG_LAUNCH_CHECK(ctx, "residual launch");
  return IEDG_OK;
}

static size_t residual_work_values(iedg_mesh mesh) {
  return (size_t)mesh->n_elem * mesh->t + 2 * (size_t)mesh->n_elem + 2 * (size_t)mesh->n_face;
}

// ---- the allocation-free residual ---------------------------------------
// File-scope device scratch of the allocation-free entry point.  In host
// code `residual_scratch` names a host-side stand-in, not device memory: the
// device address of each GPU's copy is looked up once per device (from
// iedg_create, with that device current) and only that address is used.
constexpr size_t kResidualScratchValues = size_t(2) << 20;   // 16 MiB of FP64
static __device__ __align__(256) double residual_scratch[kResidualScratchValues];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

iedg_status residual_scratch_init(iedg_context ctx) {
  const int dev = ctx->device;
  if (dev < 0 || dev >= kMaxDevices) return set_error(ctx, IEDG_ERR_UNSUPPORTED, "device %d >= %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return IEDG_OK;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(residual_scratch));
  if (e != hipSuccess || !p) return hip_check(ctx, e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
  g_scratch_ptr[dev] = static_cast<double*>(p);
  return IEDG_OK;
}

}  // namespace iedg

using namespace iedg;

extern "C" iedg_status iedg_residual_full(iedg_context ctx, iedg_mesh mesh, int32_t n_local, const double* A,
                                          const double* B, const double* C, const double* D, const double* F,
                                          const double* G, const double* z, const double* uhat, double* rF,
                                          double* rG, double* sums, hipStream_t stream) {
  if (!ctx || !mesh || !A || !B || !C || !D || !F || !G || !z || !uhat || !rF || !rG || !sums || n_local <= 0)
    return IEDG_ERR_INVALID_ARG;
  // mesh-owned scratch, allocated with the mesh
  return residual_launch(ctx, mesh, n_local, A, B, C, D, F, G, z, uhat, rF, rG, sums, mesh->d_rwork, stream);
}

extern "C" iedg_status iedg_residual_full_noalloc(iedg_context ctx, iedg_mesh mesh, int32_t n_local,
                                                  const double* A, const double* B, const double* C,
                                                  const double* D, const double* F, const double* G,
                                                  const double* z, const double* uhat, double* rF, double* rG,
                                                  double* sums, hipStream_t stream) {
  if (!ctx || !mesh || !A || !B || !C || !D || !F || !G || !z || !uhat || !rF || !rG || !sums || n_local <= 0)
    return set_error(ctx, IEDG_ERR_INVALID_ARG, "residual_full_noalloc: null argument or n <= 0");
  const size_t need = residual_work_values(mesh);
  if (need > kResidualScratchValues)
    return set_error(ctx, IEDG_ERR_UNSUPPORTED,
                     "residual_full_noalloc: needs %zu scratch values (E t + 2 E + 2 n_face), the static "
                     "scratch holds %zu", need, kResidualScratchValues);
  double* work = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (ctx->device >= 0 && ctx->device < kMaxDevices) work = g_scratch_ptr[ctx->device];
  }
  if (!work) return set_error(ctx, IEDG_ERR_HIP, "residual_full_noalloc: scratch address of device %d unknown",
                              ctx->device);
  return residual_launch(ctx, mesh, n_local, A, B, C, D, F, G, z, uhat, rF, rG, sums, work, stream);
}
