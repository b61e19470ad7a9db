// Context, error handling, mesh construction (host code of libiedg).
#include <algorithm>
#include <cstdarg>
#include <climits>
#include <set>

#include "common.h"
#include "mesh.h"

namespace iedg {

iedg_status set_error(iedg_context ctx, iedg_status s, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ctx->last_error = buf;
  }
  return s;
}

iedg_status hip_check(iedg_context ctx, hipError_t e, const char* what) {
  return set_error(ctx, IEDG_ERR_HIP, "%s failed: %s", what, hipGetErrorString(e));
}

template <typename T>
static iedg_status upload(iedg_context ctx, T** dst, const std::vector<T>& src) {
  size_t bytes = std::max<size_t>(1, src.size()) * sizeof(T);
  IEDG_HIP(ctx, hipMalloc(reinterpret_cast<void**>(dst), bytes));
  if (!src.empty()) IEDG_HIP(ctx, hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  return IEDG_OK;
}

// BSR pattern, level sets and BILU(0) schedule of a block system whose rows
// are "faces" 0 .. n_face-1 with coupling lists adj[f] (including f), in
// the elimination order m->order; uploads the pattern arrays.
iedg_status build_pattern(iedg_context ctx, iedg_mesh_s* m, const std::vector<std::vector<int>>& adj) {
  const int NF = m->n_face;
  m->pos.resize(NF);
  for (int i = 0; i < NF; ++i) m->pos[m->order[i]] = i;
  // BSR pattern in position order
  m->row_ptr.assign(NF + 1, 0);
  std::vector<int32_t>& diag_slot = m->diag_slot;
  diag_slot.assign(NF, -1);
  for (int i = 0; i < NF; ++i) {
    int f = m->order[i];
    std::vector<int> cols = adj[f];
    std::sort(cols.begin(), cols.end(), [&](int x, int y) { return m->pos[x] < m->pos[y]; });
    m->row_ptr[i + 1] = m->row_ptr[i] + (int)cols.size();
    for (int g : cols) {
      if (g == f) diag_slot[i] = (int32_t)m->col_face.size();
      m->col_face.push_back(g);
    }
  }
  m->nnzb = (int64_t)m->col_face.size();
  auto slot_of = [&](int i, int g) -> int {
    for (int s = m->row_ptr[i]; s < m->row_ptr[i + 1]; ++s)
      if (m->col_face[s] == g) return s;
    return -1;
  };
  // level sets of the lower-triangular dependency graph
  std::vector<int> level(NF, 0);
  int nlev = 0;
  for (int i = 0; i < NF; ++i) {
    int lv = 0;
    for (int s = m->row_ptr[i]; s < diag_slot[i]; ++s) lv = std::max(lv, level[m->pos[m->col_face[s]]] + 1);
    level[i] = lv;
    nlev = std::max(nlev, lv + 1);
  }
  m->n_levels = nlev;
  m->level_ptr.assign(nlev + 1, 0);
  for (int i = 0; i < NF; ++i) m->level_ptr[level[i] + 1]++;
  for (int l = 0; l < nlev; ++l) m->level_ptr[l + 1] += m->level_ptr[l];
  m->level_rows.resize(NF);
  {
    std::vector<int> fill(m->level_ptr.begin(), m->level_ptr.end() - 1);
    for (int i = 0; i < NF; ++i) m->level_rows[fill[level[i]]++] = i;
  }
  m->sweep_fused = nlev > 0;
  for (int r = nlev > 0 ? m->level_ptr[nlev - 1] : 0; r < NF; ++r) {
    const int i = m->level_rows[r];
    if (diag_slot[i] + 1 != m->row_ptr[i + 1]) m->sweep_fused = false;
  }
  // BILU(0) schedule: for row i, lower slots (i,k) in elimination order; for
  // each, the updates A_ij -= L_ik U_kj over j later than k coupled to both
  std::vector<int32_t> lptr(NF + 1, 0), lslots, uptr(1, 0), upd;
  for (int i = 0; i < NF; ++i) {
    for (int s = m->row_ptr[i]; s < diag_slot[i]; ++s) {
      int k = m->pos[m->col_face[s]];
      lslots.push_back(s);
      lslots.push_back(diag_slot[k]);
      for (int s2 = diag_slot[k] + 1; s2 < m->row_ptr[k + 1]; ++s2) {
        int j = m->col_face[s2];
        int sij = slot_of(i, j);
        if (sij >= 0) {
          upd.push_back(s2);
          upd.push_back(sij);
        }
      }
      uptr.push_back((int32_t)(upd.size() / 2));
    }
    lptr[i + 1] = (int32_t)(lslots.size() / 2);
  }
  m->n_lslots = (int64_t)lslots.size() / 2;
  m->n_updates = (int64_t)upd.size() / 2;
  iedg_status st = IEDG_OK;
  if (st == IEDG_OK) st = upload(ctx, &m->d_row_face, m->order);
  if (st == IEDG_OK) st = upload(ctx, &m->d_pos, m->pos);
  if (st == IEDG_OK) st = upload(ctx, &m->d_row_ptr, m->row_ptr);
  if (st == IEDG_OK) st = upload(ctx, &m->d_col_face, m->col_face);
  if (st == IEDG_OK) st = upload(ctx, &m->d_diag_slot, diag_slot);
  if (st == IEDG_OK) st = upload(ctx, &m->d_level_rows, m->level_rows);
  if (st == IEDG_OK) st = upload(ctx, &m->d_ilu_lptr, lptr);
  if (st == IEDG_OK) st = upload(ctx, &m->d_ilu_l, lslots);
  if (st == IEDG_OK) st = upload(ctx, &m->d_ilu_uptr, uptr);
  if (st == IEDG_OK) st = upload(ctx, &m->d_ilu_upd, upd);
  return st;
}

}  // namespace iedg

using namespace iedg;

extern "C" {

const char* iedg_status_string(iedg_status s) {
  switch (s) {
    case IEDG_OK: return "ok";
    case IEDG_ERR_INVALID_ARG: return "invalid argument";
    case IEDG_ERR_SINGULAR: return "singular pivot";
    case IEDG_ERR_NOT_CONVERGED: return "not converged";
    case IEDG_ERR_NONFINITE: return "non-finite value";
    case IEDG_ERR_OOM: return "out of device memory";
    case IEDG_ERR_HIP: return "HIP runtime error";
    case IEDG_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

iedg_status iedg_create(iedg_context* out, int device) {
  if (!out) return IEDG_ERR_INVALID_ARG;
  *out = nullptr;
  auto* ctx = new iedg_context_s();
  ctx->device = device;
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess) e = hipMalloc(&ctx->d_status, sizeof(DeviceStatus));
  if (e == hipSuccess) e = hipHostMalloc(&ctx->h_status, sizeof(DeviceStatus), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc(&ctx->h_scalars, 4096, hipHostMallocDefault);
  if (e == hipSuccess) {
    DeviceStatus init{kStatusClear};
    e = hipMemcpy(ctx->d_status, &init, sizeof(init), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    iedg_destroy(ctx);
    return IEDG_ERR_HIP;
  }
  if (residual_scratch_init(ctx) != IEDG_OK) {
    iedg_destroy(ctx);
    return IEDG_ERR_HIP;
  }
  *out = ctx;
  return IEDG_OK;
}

void iedg_destroy(iedg_context ctx) {
  if (!ctx) return;
  hipDeviceSynchronize();
  if (ctx->d_status) hipFree(ctx->d_status);
  if (ctx->h_status) hipHostFree(ctx->h_status);
  if (ctx->h_scalars) hipHostFree(ctx->h_scalars);
  delete ctx;
}

const char* iedg_last_error(iedg_context ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }

iedg_status iedg_sync_status(iedg_context ctx, hipStream_t stream, int64_t* bad_index) {
  if (!ctx) return IEDG_ERR_INVALID_ARG;
  IEDG_HIP(ctx, hipMemcpyAsync(ctx->h_status, ctx->d_status, sizeof(DeviceStatus), hipMemcpyDeviceToHost, stream));
  IEDG_HIP(ctx, hipStreamSynchronize(stream));
  const DeviceStatus st = *ctx->h_status;
  const bool failed = st.word != kStatusClear;
  const int32_t code = failed ? -static_cast<int32_t>(st.word & 0xff) : 0;
  const long long index = failed ? static_cast<long long>(st.word >> 8) : -1;
  if (bad_index) *bad_index = index;
  if (failed) {
    DeviceStatus init{kStatusClear};
    IEDG_HIP(ctx, hipMemcpy(ctx->d_status, &init, sizeof(init), hipMemcpyHostToDevice));
    return set_error(ctx, static_cast<iedg_status>(code), "device reported %s at index %lld",
                     iedg_status_string(static_cast<iedg_status>(code)), index);
  }
  return IEDG_OK;
}

}  // extern "C"

namespace iedg {

// Mesh of E elements that each list S trace units of b dofs (t = S b).
static iedg_status mesh_create_general(iedg_context ctx, int E, int S, int NF, int b, const int32_t* eu,
                                       int ordering, const int32_t* order_in, iedg_mesh* out) {
  if ((int64_t)E * S * S > INT32_MAX)
    return set_error(ctx, IEDG_ERR_UNSUPPORTED, "mesh_create: E S^2 = %lld exceeds int32", (long long)E * S * S);
  // P_e^T sources of every unit, ascending (e, a)
  std::vector<int32_t> src_ptr(NF + 1, 0), src_list((size_t)E * S);
  for (int e = 0; e < E; ++e)
    for (int a = 0; a < S; ++a) {
      const int u = eu[(size_t)S * e + a];
      if (u < 0 || u >= NF) return set_error(ctx, IEDG_ERR_INVALID_ARG, "mesh_create: unit id %d out of range", u);
      src_ptr[u + 1]++;
    }
  for (int u = 0; u < NF; ++u) {
    if (src_ptr[u + 1] == 0) return set_error(ctx, IEDG_ERR_INVALID_ARG, "mesh_create: unit %d has no element", u);
    src_ptr[u + 1] += src_ptr[u];
  }
  {
    std::vector<int32_t> fill(src_ptr.begin(), src_ptr.end() - 1);
    for (int e = 0; e < E; ++e)
      for (int a = 0; a < S; ++a) src_list[fill[eu[(size_t)S * e + a]]++] = e * S + a;
  }
  // coupled units (pattern): units of a common element, sorted by id
  std::vector<std::vector<int>> adj(NF);
  {
    std::vector<int> us;
    for (int e = 0; e < E; ++e) {
      us.assign(eu + (size_t)S * e, eu + (size_t)S * (e + 1));
      std::sort(us.begin(), us.end());
      us.erase(std::unique(us.begin(), us.end()), us.end());
      for (int u : us) adj[u].insert(adj[u].end(), us.begin(), us.end());
    }
    for (auto& v : adj) {
      std::sort(v.begin(), v.end());
      v.erase(std::unique(v.begin(), v.end()), v.end());
    }
  }
  auto* m = new iedg_mesh_s();
  m->ctx = ctx;
  m->n_elem = E;
  m->n_face = NF;
  m->b = b;
  m->slots = S;
  m->t = S * b;
  m->n_trace = int64_t(NF) * b;
  // ordering
  m->order.resize(NF);
  if (ordering == 1) {
    for (int f = 0; f < NF; ++f) m->order[f] = f;
  } else if (ordering == 2) {
    if (!order_in) { delete m; return set_error(ctx, IEDG_ERR_INVALID_ARG, "mesh_create: ordering 2 needs order"); }
    std::vector<char> seen(NF, 0);
    for (int i = 0; i < NF; ++i) {
      int f = order_in[i];
      if (f < 0 || f >= NF || seen[f]) { delete m; return set_error(ctx, IEDG_ERR_INVALID_ARG, "mesh_create: order is not a permutation"); }
      seen[f] = 1;
      m->order[i] = f;
    }
  } else if (ordering == 0) {
    // greedy colouring: ascending unit id, smallest colour not used by an
    // already coloured coupled unit; rows listed by (colour, unit id)
    std::vector<int> colour(NF, -1);
    int ncol = 0;
    for (int f = 0; f < NF; ++f) {
      std::vector<char> used(adj[f].size() + 1, 0);
      for (int g : adj[f])
        if (g != f && colour[g] >= 0 && colour[g] < (int)used.size()) used[colour[g]] = 1;
      int c = 0;
      while (used[c]) ++c;
      colour[f] = c;
      ncol = std::max(ncol, c + 1);
    }
    int i = 0;
    for (int c = 0; c < ncol; ++c)
      for (int f = 0; f < NF; ++f)
        if (colour[f] == c) m->order[i++] = f;
  } else {
    delete m;
    return set_error(ctx, IEDG_ERR_INVALID_ARG, "mesh_create: unknown ordering %d", ordering);
  }
  iedg_status st = build_pattern(ctx, m, adj);
  if (st != IEDG_OK) {
    iedg_mesh_destroy(m);
    return st;
  }
  // assembly lists: block (u_a, u_c) receives Ke_e[a][c]; the block of a
  // pair is found by bisection over its row's columns (sorted by position)
  std::vector<int32_t> slot_of((size_t)E * S * S);
  for (int e = 0; e < E; ++e)
    for (int a = 0; a < S; ++a) {
      const int i = m->pos[eu[(size_t)S * e + a]];
      const int r0 = m->row_ptr[i], r1 = m->row_ptr[i + 1];
      for (int c = 0; c < S; ++c) {
        const int pc = m->pos[eu[(size_t)S * e + c]];
        int lo = r0, hi = r1;
        while (lo < hi) {
          const int mid = (lo + hi) / 2;
          if (m->pos[m->col_face[mid]] < pc) lo = mid + 1;
          else hi = mid;
        }
        slot_of[((size_t)e * S + a) * S + c] = lo;
      }
    }
  std::vector<int32_t> asm_ptr(m->nnzb + 1, 0), asm_list((size_t)E * S * S);
  for (int32_t sl : slot_of) asm_ptr[sl + 1]++;
  for (int64_t s = 0; s < m->nnzb; ++s) asm_ptr[s + 1] += asm_ptr[s];
  {
    std::vector<int32_t> fill(asm_ptr.begin(), asm_ptr.end() - 1);
    for (size_t code = 0; code < slot_of.size(); ++code) asm_list[fill[slot_of[code]]++] = (int32_t)code;
  }
  std::vector<int32_t> ef(eu, eu + (size_t)S * E);
  if (st == IEDG_OK) st = upload(ctx, &m->d_elem_faces, ef);
  if (st == IEDG_OK) st = upload(ctx, &m->d_asm_ptr, asm_ptr);
  if (st == IEDG_OK) st = upload(ctx, &m->d_asm_list, asm_list);
  if (st == IEDG_OK) st = upload(ctx, &m->d_src_ptr, src_ptr);
  if (st == IEDG_OK) st = upload(ctx, &m->d_src_list, src_list);
  if (st == IEDG_OK) {
    const size_t rw = (size_t)E * m->t + 2 * (size_t)E + 2 * (size_t)NF;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&m->d_rwork), rw * sizeof(double));
    if (e != hipSuccess) st = set_error(ctx, IEDG_ERR_OOM, "mesh residual scratch: %s", hipGetErrorString(e));
  }
  if (st != IEDG_OK) {
    iedg_mesh_destroy(m);
    return st;
  }
  *out = m;
  return IEDG_OK;
}

}  // namespace iedg

extern "C" {

iedg_status iedg_mesh_create(iedg_context ctx, int32_t n_elem, int32_t n_face, int32_t face_dofs,
                             const int32_t* elem_faces, int32_t ordering, const int32_t* order_in,
                             iedg_mesh* out) {
  if (!ctx || !out || !elem_faces || n_elem <= 0 || n_face <= 0 || face_dofs <= 0)
    return set_error(ctx, IEDG_ERR_INVALID_ARG, "mesh_create: bad arguments");
  if (face_dofs > 128)
    return set_error(ctx, IEDG_ERR_UNSUPPORTED, "mesh_create: face_dofs %d > 128", face_dofs);
  *out = nullptr;
  // faces: listed at most once by an element, by at most two elements
  std::vector<int> count(n_face, 0);
  for (int e = 0; e < n_elem; ++e)
    for (int a = 0; a < 6; ++a) {
      const int f = elem_faces[6 * e + a];
      if (f < 0 || f >= n_face) return set_error(ctx, IEDG_ERR_INVALID_ARG, "mesh_create: face id %d out of range", f);
      for (int a2 = 0; a2 < a; ++a2)
        if (elem_faces[6 * e + a2] == f)
          return set_error(ctx, IEDG_ERR_INVALID_ARG, "mesh_create: element %d lists face %d twice", e, f);
      if (++count[f] > 2)
        return set_error(ctx, IEDG_ERR_INVALID_ARG, "mesh_create: face %d shared by more than two elements", f);
    }
  return mesh_create_general(ctx, n_elem, 6, n_face, face_dofs, elem_faces, ordering, order_in, out);
}

iedg_status iedg_mesh_create_slots(iedg_context ctx, int32_t n_elem, int32_t slots, int32_t n_units,
                                   int32_t unit_dofs, const int32_t* elem_units, int32_t ordering,
                                   const int32_t* order_in, iedg_mesh* out) {
  if (!ctx || !out || !elem_units || n_elem <= 0 || slots <= 0 || n_units <= 0 || unit_dofs <= 0)
    return set_error(ctx, IEDG_ERR_INVALID_ARG, "mesh_create_slots: bad arguments");
  if (unit_dofs > 128)
    return set_error(ctx, IEDG_ERR_UNSUPPORTED, "mesh_create_slots: unit_dofs %d > 128", unit_dofs);
  *out = nullptr;
  return mesh_create_general(ctx, n_elem, slots, n_units, unit_dofs, elem_units, ordering, order_in, out);
}

void iedg_mesh_destroy(iedg_mesh m) {
  if (!m) return;
  int32_t* ptrs[] = {m->d_elem_faces, m->d_row_face, m->d_pos, m->d_row_ptr, m->d_col_face,
                     m->d_diag_slot, m->d_level_rows, m->d_asm_ptr, m->d_asm_list, m->d_src_ptr, m->d_src_list,
                     m->d_ilu_lptr, m->d_ilu_l, m->d_ilu_uptr, m->d_ilu_upd};
  for (int32_t* p : ptrs)
    if (p) hipFree(p);
  if (m->d_rwork) hipFree(m->d_rwork);
  delete m;
}

iedg_status iedg_mesh_query(iedg_mesh m, iedg_mesh_info* info, int32_t* order, int32_t* level_ptr,
                            int32_t* row_ptr, int32_t* col_face) {
  if (!m) return IEDG_ERR_INVALID_ARG;
  if (info) {
    info->n_elem = m->n_elem;
    info->n_face = m->n_face;
    info->face_dofs = m->b;
    info->n_trace = m->n_trace;
    info->nnzb = m->nnzb;
    info->n_levels = m->n_levels;
  }
  if (order) std::copy(m->order.begin(), m->order.end(), order);
  if (level_ptr) std::copy(m->level_ptr.begin(), m->level_ptr.end(), level_ptr);
  if (row_ptr) std::copy(m->row_ptr.begin(), m->row_ptr.end(), row_ptr);
  if (col_face) std::copy(m->col_face.begin(), m->col_face.end(), col_face);
  return IEDG_OK;
}

}  // extern "C"
