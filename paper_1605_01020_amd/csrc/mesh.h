// Trace mesh: block pattern of K, element->BSR scatter map, BILU(0) schedule.
#pragma once

#include "common.h"

// Rows ("faces" below) are the trace units: faces with private dofs, or the
// nodes of the IEDG numbering; element e lists `slots` units, t = slots b.
struct iedg_mesh_s {
  iedg_context ctx = nullptr;
  int32_t n_elem = 0, n_face = 0, b = 0, t = 0, slots = 6;
  int64_t n_trace = 0, nnzb = 0;
  int32_t n_levels = 0;
  // the rows of the last level have no upper slots (true for every
  // symmetric pattern): the BILU(0) apply then runs that level's forward and
  // backward steps in one launch
  bool sweep_fused = false;
  int64_t n_lslots = 0, n_updates = 0;

  // host copies (exported by iedg_mesh_query)
  std::vector<int32_t> order;       // row i -> face
  std::vector<int32_t> pos;         // face -> row
  std::vector<int32_t> level_ptr;   // [n_levels + 1] into level_rows
  std::vector<int32_t> level_rows;  // rows grouped by level, ascending within a level
  std::vector<int32_t> row_ptr;     // [n_face + 1]
  std::vector<int32_t> col_face;    // [nnzb]
  std::vector<int32_t> diag_slot;   // [n_face]

  // device copies
  int32_t* d_elem_faces = nullptr;  // [E][slots]: unit of each local slot
  int32_t* d_row_face = nullptr;    // [n_face]
  int32_t* d_pos = nullptr;         // [n_face]: face -> row
  int32_t* d_row_ptr = nullptr;     // [n_face + 1]
  int32_t* d_col_face = nullptr;    // [nnzb]
  int32_t* d_diag_slot = nullptr;   // [n_face]
  int32_t* d_level_rows = nullptr;  // [n_face]
  // assembly of K: block s receives Ke_e[a][c] for every code e*S*S + a*S + c
  // in asm_list[asm_ptr[s] .. asm_ptr[s+1]) (ascending: e, then a, then c)
  int32_t* d_asm_ptr = nullptr;     // [nnzb + 1]
  int32_t* d_asm_list = nullptr;    // [E * slots^2]
  // P_e^T: unit u receives slot a of element e for every code e*S + a in
  // src_list[src_ptr[u] .. src_ptr[u+1]) (ascending)
  int32_t* d_src_ptr = nullptr;     // [n_face + 1]
  int32_t* d_src_list = nullptr;    // [E * slots]
  int32_t* d_ilu_lptr = nullptr;    // [n_face + 1] into ilu_l (per row)
  int32_t* d_ilu_l = nullptr;       // [n_lslots][2]: slot (i,k), diag slot of k
  int32_t* d_ilu_uptr = nullptr;    // [n_lslots + 1] into ilu_upd
  int32_t* d_ilu_upd = nullptr;     // [n_updates][2]: slot (k,j), slot (i,j)

  // scratch of the FP64 residual (q [E][t], partial sums 2E + 2 n_face),
  // owned by the mesh so that residual launches never allocate
  double* d_rwork = nullptr;
};

namespace iedg {
// Pattern, level sets and BILU(0) schedule of rows 0 .. m->n_face-1 with
// coupling lists adj (each including the row itself), in the order
// m->order; uploads the pattern arrays (context.hip).
iedg_status build_pattern(iedg_context ctx, iedg_mesh_s* m, const std::vector<std::vector<int>>& adj);
// The global mesh a RAS preconditioner was built on (ras.hip).
iedg_mesh ras_mesh(iedg_ras r);
}  // namespace iedg
