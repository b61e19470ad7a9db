// Restricted additive Schwarz preconditioner with delta-level overlap and
// BILU(0) subdomain solves (section 2.2.2, RAS equation), emulated on one
// GPU: M^{-1} x = sum_i R_i^0 BILU(0)(K_i)^{-1} R_i^delta x.
//
// The N overlapped subdomain systems K_i = K restricted to S_i^delta are
// held together as one block-sparse "local" system whose rows are the
// (subdomain, face) pairs, subdomain-major and, within a subdomain, in the
// elimination order of the global mesh.  Subdomains share no couplings in
// it, so the BILU(0) factorisation and the level-scheduled sweeps of the
// global system apply unchanged (independent subdomains fall into the same
// levels).  An application is: gather x onto the local rows (R_i^delta),
// the two sweeps, and a scatter that writes every face from the copy of
// its own subdomain (R_i^0).
#include <algorithm>
#include <vector>

#include "common.h"
#include "mesh.h"

struct iedg_ras_s {
  iedg_context ctx = nullptr;
  iedg_mesh gmesh = nullptr;
  iedg_mesh_s* lmesh = nullptr;     // the local system (no elements)
  int n_sub = 0, delta = 0;
  int32_t* d_gface = nullptr;       // [n_loc]: global face of each local row
  int32_t* d_owner = nullptr;       // [n_face]: local row holding a face's own copy
  int32_t* d_gslot = nullptr;       // [nnzb_loc]: global BSR slot of each local block
  double* d_x = nullptr;            // [n_loc * b]
  double* d_y = nullptr;            // [n_loc * b]
};

namespace iedg {

// xl[r*b + l] = x[gface[r]*b + l]
__global__ void ras_gather_kernel(int64_t n, int b, const int32_t* gface, const double* x, double* xl,
                                  const int* skip) {
  if (skip && *skip) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t r = i / b, l = i % b;
  xl[i] = x[(int64_t)gface[r] * b + l];
}

// y[f*b + l] = yl[owner[f]*b + l]
__global__ void ras_scatter_kernel(int64_t n, int b, const int32_t* owner, const double* yl, double* y,
                                   const int* skip) {
  if (skip && *skip) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t f = i / b, l = i % b;
  y[i] = yl[(int64_t)owner[f] * b + l];
}

// Mloc[s] = K[gslot[s]] (b x b blocks), one workgroup per local block.
template <typename T>
__global__ __launch_bounds__(256) void ras_block_gather_kernel(int b, const int32_t* gslot, const T* K, T* M) {
  const int64_t s = blockIdx.x;
  const size_t bb = (size_t)b * b;
  const T* src = K + (size_t)gslot[s] * bb;
  T* dst = M + (size_t)s * bb;
  for (int q = threadIdx.x; q < (int)bb; q += 256) dst[q] = src[q];
}

iedg_status ilu0_apply_launch(iedg_context ctx, iedg_mesh m, iedg_prec mprec, const void* M, const double* x,
                              double* y, hipStream_t stream, const int* skip);

iedg_status ras_apply_launch(iedg_context ctx, iedg_ras ras, iedg_prec mprec, const void* Mloc, const double* x,
                             double* y, hipStream_t stream, const int* skip) {
  const int b = ras->gmesh->b;
  const int64_t nl = ras->lmesh->n_trace, ng = ras->gmesh->n_trace;
  hipLaunchKernelGGL(ras_gather_kernel, dim3((unsigned)((nl + 255) / 256)), dim3(256), 0, stream, nl, b,
                     ras->d_gface, x, ras->d_x, skip);
  iedg_status s = ilu0_apply_launch(ctx, ras->lmesh, mprec, Mloc, ras->d_x, ras->d_y, stream, skip);
  if (s != IEDG_OK) return s;
  hipLaunchKernelGGL(ras_scatter_kernel, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, stream, ng, b,
                     ras->d_owner, ras->d_y, y, skip);
  IEDG_LAUNCH_CHECK(ctx, "ras apply launch");
  return IEDG_OK;
}

iedg_mesh ras_mesh(iedg_ras r) { return r->gmesh; }

template <typename T>
static iedg_status upload_vec(iedg_context ctx, T** dst, const std::vector<T>& src) {
  IEDG_HIP(ctx, hipMalloc(reinterpret_cast<void**>(dst), std::max<size_t>(1, src.size()) * sizeof(T)));
  if (!src.empty()) IEDG_HIP(ctx, hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  return IEDG_OK;
}

}  // namespace iedg

using namespace iedg;

extern "C" void iedg_ras_destroy(iedg_ras r) {
  if (!r) return;
  if (r->lmesh) iedg_mesh_destroy(r->lmesh);
  int32_t* ip[] = {r->d_gface, r->d_owner, r->d_gslot};
  for (int32_t* p : ip)
    if (p) (void)hipFree(p);
  if (r->d_x) (void)hipFree(r->d_x);
  if (r->d_y) (void)hipFree(r->d_y);
  delete r;
}

extern "C" iedg_status iedg_ras_create(iedg_context ctx, iedg_mesh mesh, int32_t n_sub, const int32_t* part,
                                       int32_t delta, iedg_ras* out) {
  if (!ctx || !mesh || !part || !out || n_sub < 1 || delta < 0)
    return set_error(ctx, IEDG_ERR_INVALID_ARG, "ras_create: bad arguments");
  *out = nullptr;
  const int NF = mesh->n_face;
  std::vector<int> count(n_sub, 0);
  for (int f = 0; f < NF; ++f) {
    if (part[f] < 0 || part[f] >= n_sub)
      return set_error(ctx, IEDG_ERR_INVALID_ARG, "ras_create: part[%d] = %d outside [0, %d)", f, part[f], n_sub);
    count[part[f]]++;
  }
  for (int i = 0; i < n_sub; ++i)
    if (!count[i]) return set_error(ctx, IEDG_ERR_INVALID_ARG, "ras_create: subdomain %d has no face", i);
  // coupled faces of each face (the pattern of K)
  auto cols = [&](int f, auto&& fn) {
    const int r = mesh->pos[f];
    for (int s = mesh->row_ptr[r]; s < mesh->row_ptr[r + 1]; ++s) fn(mesh->col_face[s], s);
  };
  // local rows: subdomain-major, global elimination order within a subdomain
  std::vector<int32_t> gface, owner(NF, -1), sub_of;
  std::vector<std::vector<int>> adj;
  std::vector<int> lrow(NF, -1), mark(NF, 0);
  for (int i = 0; i < n_sub; ++i) {
    std::vector<int> Sd;
    for (int f = 0; f < NF; ++f)
      if (part[f] == i) { Sd.push_back(f); mark[f] = 1; }
    size_t frontier = 0;
    for (int d = 0; d < delta; ++d) {
      const size_t end = Sd.size();
      for (size_t q = frontier; q < end; ++q)
        cols(Sd[q], [&](int g, int) {
          if (!mark[g]) { mark[g] = 1; Sd.push_back(g); }
        });
      frontier = end;
    }
    std::sort(Sd.begin(), Sd.end(), [&](int x, int y) { return mesh->pos[x] < mesh->pos[y]; });
    const int base = (int)gface.size();
    for (size_t q = 0; q < Sd.size(); ++q) {
      lrow[Sd[q]] = base + (int)q;
      gface.push_back(Sd[q]);
      sub_of.push_back(i);
      if (part[Sd[q]] == i) owner[Sd[q]] = base + (int)q;
    }
    for (int f : Sd) {
      std::vector<int> a;
      cols(f, [&](int g, int) {
        if (lrow[g] >= 0) a.push_back(lrow[g]);
      });
      adj.push_back(std::move(a));
    }
    for (int f : Sd) { lrow[f] = -1; mark[f] = 0; }
  }
  const int NL = (int)gface.size();
  auto* r = new iedg_ras_s();
  r->ctx = ctx;
  r->gmesh = mesh;
  r->n_sub = n_sub;
  r->delta = delta;
  auto* lm = new iedg_mesh_s();
  r->lmesh = lm;
  lm->ctx = ctx;
  lm->n_elem = 0;
  lm->n_face = NL;
  lm->b = mesh->b;
  lm->t = mesh->t;
  lm->n_trace = (int64_t)NL * mesh->b;
  lm->order.resize(NL);
  for (int q = 0; q < NL; ++q) lm->order[q] = q;
  iedg_status st = build_pattern(ctx, lm, adj);
  // global slot of every local block
  std::vector<int32_t> gslot(lm->nnzb, -1);
  if (st == IEDG_OK) {
    for (int q = 0; q < NL; ++q) {
      const int f = gface[q];
      for (int s = lm->row_ptr[q]; s < lm->row_ptr[q + 1]; ++s) {
        const int g = gface[lm->col_face[s]];
        cols(f, [&](int gg, int gs) {
          if (gg == g) gslot[s] = gs;
        });
        if (gslot[s] < 0) { st = set_error(ctx, IEDG_ERR_INVALID_ARG, "ras_create: pattern mismatch"); break; }
      }
      if (st != IEDG_OK) break;
    }
  }
  if (st == IEDG_OK) st = upload_vec(ctx, &r->d_gface, gface);
  if (st == IEDG_OK) st = upload_vec(ctx, &r->d_owner, owner);
  if (st == IEDG_OK) st = upload_vec(ctx, &r->d_gslot, gslot);
  if (st == IEDG_OK) {
    const size_t nv = std::max<size_t>(1, (size_t)lm->n_trace);
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&r->d_x), nv * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&r->d_y), nv * sizeof(double));
    if (e != hipSuccess) st = set_error(ctx, IEDG_ERR_OOM, "ras_create: local vectors");
  }
  if (st != IEDG_OK) {
    iedg_ras_destroy(r);
    return st;
  }
  *out = r;
  return IEDG_OK;
}

extern "C" iedg_status iedg_ras_query(iedg_ras r, iedg_ras_info* info) {
  if (!r || !info) return IEDG_ERR_INVALID_ARG;
  info->n_sub = r->n_sub;
  info->delta = r->delta;
  info->n_local_rows = r->lmesh->n_face;
  info->nnzb = r->lmesh->nnzb;
  info->n_levels = r->lmesh->n_levels;
  return IEDG_OK;
}

extern "C" iedg_status iedg_ras_factor(iedg_context ctx, iedg_ras r, iedg_prec prec, const void* Kbsr, void* Mloc,
                                       hipStream_t stream) {
  if (!ctx || !r || !Kbsr || !Mloc) return set_error(ctx, IEDG_ERR_INVALID_ARG, "ras_factor: null argument");
  if (prec != IEDG_F64 && prec != IEDG_F32 && prec != IEDG_BF16)
    return set_error(ctx, IEDG_ERR_INVALID_ARG, "ras_factor: precision %d", (int)prec);
  const unsigned nb = (unsigned)r->lmesh->nnzb;
  if (prec == IEDG_F64)
    hipLaunchKernelGGL(ras_block_gather_kernel<double>, dim3(nb), dim3(256), 0, stream, r->gmesh->b, r->d_gslot,
                       (const double*)Kbsr, (double*)Mloc);
  else
    hipLaunchKernelGGL(ras_block_gather_kernel<float>, dim3(nb), dim3(256), 0, stream, r->gmesh->b, r->d_gslot,
                       (const float*)Kbsr, (float*)Mloc);
  IEDG_LAUNCH_CHECK(ctx, "ras block gather");
  return iedg_factor_ilu0(ctx, r->lmesh, prec, Mloc, Mloc, stream);
}

extern "C" iedg_status iedg_ras_apply(iedg_context ctx, iedg_ras r, iedg_prec prec, const void* Mloc,
                                      const double* x, double* y, hipStream_t stream) {
  if (!ctx || !r || !Mloc || !x || !y) return set_error(ctx, IEDG_ERR_INVALID_ARG, "ras_apply: null argument");
  return ras_apply_launch(ctx, r, prec, Mloc, x, y, stream, nullptr);
}
