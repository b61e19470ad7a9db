/*
 * iedg.h -- C ABI of the MI355X (gfx950) library for the linear solve of one
 * Newton step of an IEDG discretisation.
 *
 * Paper: Fernandez, Nguyen, Roca, Peraire, "Implicit large-eddy simulation
 * of compressible flows using the Interior Embedded Discontinuous Galerkin
 * method", section 2.2.  The Newton linear system of section 2.2.1 is
 *
 *     [ A  B ] [ dZ ]   [ F ]
 *     [ C  D ] [ dU ] = [ G ]
 *
 * with A block diagonal (one dense block per element).  Eliminating dZ gives
 * the trace system K dU = R, K = D - C A^{-1} B, R = G - C A^{-1} F (eq. LS),
 * which is solved by restarted GMRES with iterated classical Gram-Schmidt,
 * left-preconditioned by the zero-fill block ILU of K (section 2.2.2,
 * eq. LS1).  dZ is then recovered element by element.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Sizes: n = local (q, u) dofs per element, b = trace dofs per face,
 *   t = 6 b trace dofs per element (faces in local order -x,+x,-y,+y,-z,+z),
 *   E elements, N_f faces, N_t = N_f b global trace dofs (dof f*b + l).
 * - Every array argument is a DEVICE pointer owned by the caller unless the
 *   argument says "host".  Dense element blocks are row-major and
 *   element-major: X[e][row][col].  Global trace vectors are FP64 [N_t].
 * - Calls enqueue work on the given HIP stream and return at once, except
 *   where a call says it synchronises.  Argument errors are returned
 *   immediately (nothing is enqueued).  Conditions detected on the device
 *   (a zero or non-finite pivot) are latched in a device status word and
 *   reported by iedg_sync_status().
 * - Hot calls do not allocate.  Device memory the library needs beyond the
 *   caller's arrays is allocated when an object is created (context, mesh,
 *   GMRES state, batch plan) and freed when it is destroyed.
 * - A context is not thread-safe; use one per host thread.
 */
#ifndef IEDG_H
#define IEDG_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  IEDG_OK = 0,
  IEDG_ERR_INVALID_ARG = -1,   /* bad size, null pointer, aliasing, etc. */
  IEDG_ERR_SINGULAR = -2,      /* zero / non-finite pivot met on the device */
  IEDG_ERR_NOT_CONVERGED = -3, /* GMRES hit max_iters above tolerance */
  IEDG_ERR_NONFINITE = -4,     /* NaN/Inf in a right-hand side or residual */
  IEDG_ERR_OOM = -5,           /* workspace allocation failed */
  IEDG_ERR_HIP = -6,           /* a HIP runtime call failed */
  IEDG_ERR_UNSUPPORTED = -7    /* size or precision not built in */
} iedg_status;

/* Storage / arithmetic precision of factors and assembled blocks.
 * IEDG_F64: FP64 storage and MFMA arithmetic.
 * IEDG_F32: FP32 storage, FP32 MFMA with FP32 accumulation.
 * IEDG_BF16: FP32 storage; trailing updates of the condensation take BF16
 *            operands with FP32 accumulation (MFMA); panels stay FP32. */
typedef enum { IEDG_F64 = 0, IEDG_F32 = 1, IEDG_BF16 = 2 } iedg_prec;

typedef struct iedg_context_s* iedg_context;
typedef struct iedg_mesh_s* iedg_mesh;

/* ---- context ---------------------------------------------------------- */
iedg_status iedg_create(iedg_context* out, int device);
void iedg_destroy(iedg_context ctx);
const char* iedg_last_error(iedg_context ctx);
const char* iedg_status_string(iedg_status s);
/* Synchronises `stream`, then returns and clears the device status word:
 * IEDG_OK or IEDG_ERR_SINGULAR; *bad_index (may be NULL) receives the index
 * of the first failing element (condense) or block row (factor_ilu0). */
iedg_status iedg_sync_status(iedg_context ctx, hipStream_t stream, int64_t* bad_index);

/* ---- trace mesh and block pattern ------------------------------------- */
/* Builds the block sparsity pattern of K (a b x b block (f, g) exists iff
 * faces f and g belong to a common element; section 2.2.1), the element ->
 * BSR scatter map, the row ordering used by BILU(0) and its level sets
 * (section 2.2.2), and copies them to the device.
 * elem_faces: host [n_elem][6] face ids, local order -x,+x,-y,+y,-z,+z.
 * ordering: 0 = greedy colouring (faces visited by ascending id, each takes
 *   the smallest colour unused by an already coloured face sharing an
 *   element; rows listed by (colour, face id)); 1 = natural face order;
 *   2 = the permutation given in `order` (host [n_face]), e.g. the minimum
 *   discarded fill order from iedg_mdf_order.
 * BSR layout: block row i (0 <= i < n_face) is face order[i]; its blocks
 * occupy slots row_ptr[i] .. row_ptr[i+1]-1, sorted by the position of their
 * column face in the ordering (so lower blocks, the diagonal, then upper
 * blocks).  A block is b*b contiguous values stored COLUMN-major (entry
 * (r, c) at c*b + r). */
iedg_status iedg_mesh_create(iedg_context ctx, int32_t n_elem, int32_t n_face,
                             int32_t face_dofs, const int32_t* elem_faces,
                             int32_t ordering, const int32_t* order,
                             iedg_mesh* out);
/* The same for any trace numbering (section 2.1): element e lists `slots`
 * trace units (elem_units host [n_elem][slots]) of unit_dofs dofs each (unit
 * u holds dofs u * unit_dofs .. + unit_dofs - 1; the element's t = slots *
 * unit_dofs local trace dofs are its slots' dofs in slot order).  An element
 * may list a unit in several slots: the IEDG numbering, whose units are
 * trace nodes of m components shared along interior faces, does where an
 * element's own faces meet.  K has a block (u, w) iff u and w appear in a
 * common element; the block receives Ke_e[a][c] for every element e and
 * slots a, c mapping to u, w (ascending e, a, c), and P_e^T adds every local
 * dof into its unit's dof (ascending e, a).  unit_dofs <= 128; every unit
 * must appear in an element (IEDG_ERR_INVALID_ARG otherwise).  ordering and
 * layout as for iedg_mesh_create, with units in place of faces;
 * iedg_mesh_create is this call with slots = 6 and face checks (a face is
 * listed once by an element and by at most two elements). */
iedg_status iedg_mesh_create_slots(iedg_context ctx, int32_t n_elem, int32_t slots,
                                   int32_t n_units, int32_t unit_dofs,
                                   const int32_t* elem_units, int32_t ordering,
                                   const int32_t* order, iedg_mesh* out);
void iedg_mesh_destroy(iedg_mesh mesh);

typedef struct {
  int64_t n_elem, n_face, face_dofs, n_trace, nnzb, n_levels;
} iedg_mesh_info;
/* Host outputs, each may be NULL: order [n_face], level_ptr [n_levels+1]
 * (rows level_ptr[l] .. level_ptr[l+1]-1 of the ordering form level l),
 * row_ptr [n_face+1], col_face [nnzb]. */
iedg_status iedg_mesh_query(iedg_mesh mesh, iedg_mesh_info* info, int32_t* order,
                            int32_t* level_ptr, int32_t* row_ptr, int32_t* col_face);

/* ---- a1: element static condensation (section 2.2.1, eq. LS) ---------- */
/* For every element, with the bordered matrix [A B F; C D 0]:
 *   P A = L U (partial pivoting over the rows of A),
 *   U12 = L^{-1} P B,  w = L^{-1} P F,  L21 = C U^{-1},
 *   Ke = D - L21 U12 = D - C A^{-1} B,  r = -L21 w = -C A^{-1} F.
 * Inputs (FP64, read only): A [E][n][n], B [E][n][t], C [E][t][n],
 *   D [E][t][t], F [E][n] (F may be NULL: then w and r are not written).
 * Outputs (element type given by prec: double for IEDG_F64, float
 *   otherwise): LU [E][n][n], U12 [E][n][t], L21 [E][t][n], Ke [E][t][t];
 *   perm [E][n] int32 (row i of P A is row perm[i] of A); w [E][n] and
 *   r [E][t] FP64.  Row interchanges are not applied to the stored rows:
 *   row i of the packed factors of P A (unit-lower L below the diagonal,
 *   U on and above) is stored in row perm[i] of LU, and likewise row i of
 *   U12 and entry i of w sit in row perm[i] (the row of A they came from).
 *   L21, Ke and r are indexed by the rows of C.
 * Outputs must not overlap inputs.  A zero or non-finite pivot latches
 * IEDG_ERR_SINGULAR with the element index.
 * Limits: n a multiple of 4 and at most 2560, t even and at most 1024
 * (IEDG_ERR_UNSUPPORTED otherwise); every array 16-byte aligned, as device
 * allocators return it (IEDG_ERR_INVALID_ARG otherwise). */
iedg_status iedg_condense(iedg_context ctx, int32_t n_elem, int32_t n_local,
                          int32_t n_trace_elem, iedg_prec prec,
                          const double* A, const double* B, const double* C,
                          const double* D, const double* F,
                          void* LU, int32_t* perm, void* U12, void* L21,
                          double* w, void* Ke, double* r, hipStream_t stream);

/* Right-hand-side-only condensation with retained factors (section 2.2.1):
 * w = L^{-1} P F and r = -L21 w per element, w stored in the same row
 * order as iedg_condense writes it.  LU, perm, L21 as written by
 * iedg_condense (`prec` storage). */
iedg_status iedg_condense_rhs(iedg_context ctx, int32_t n_elem, int32_t n_local,
                              int32_t n_trace_elem, iedg_prec prec,
                              const void* LU, const int32_t* perm, const void* L21,
                              const double* F, double* w, double* r,
                              hipStream_t stream);

/* Batched condensation (section 2.2.1, eq. LS) of several meshes (segments)
 * in one persistent launch: one workgroup per CU slot takes (segment,
 * element) items from a device queue until it is empty.  Each item is
 * computed exactly as iedg_condense computes it (bitwise the same outputs,
 * with the sub-panel width the context held for that size when the plan was
 * made).  Segments may differ in element size (iedg_batch_create_sized:
 * n_local[s], n_trace_elem[s] per segment, each a size iedg_condense
 * accepts); the work list starts with the largest elements and interleaves
 * the segments of one size.  The plan copies the segment table and work list
 * to the device once; iedg_condense_batched only launches (a reset kernel
 * and the condensation; it can be captured in a HIP graph).  Calls with one
 * plan must not overlap (they share the queue counter).  Segment pointers
 * must stay valid for the plan's lifetime.  iedg_batch_create is the
 * one-size form.  Errors: IEDG_ERR_INVALID_ARG (sizes, null or unaligned
 * arrays of a segment with elements), IEDG_ERR_UNSUPPORTED (size or
 * precision), IEDG_ERR_HIP / IEDG_ERR_OOM from the uploads. */
typedef struct {
  int32_t n_elem;
  const double *A, *B, *C, *D, *F;
  void* LU;
  int32_t* perm;
  void *U12, *L21;
  double* w;
  void* Ke;
  double* r;
} iedg_condense_segment;
typedef struct iedg_batch_s* iedg_batch;
iedg_status iedg_batch_create(iedg_context ctx, int32_t n_seg, const iedg_condense_segment* segs,
                              int32_t n_local, int32_t n_trace_elem, iedg_prec prec,
                              iedg_batch* out);
iedg_status iedg_batch_create_sized(iedg_context ctx, int32_t n_seg, const iedg_condense_segment* segs,
                                    const int32_t* n_local /* host, [n_seg] */,
                                    const int32_t* n_trace_elem /* host, [n_seg] */, iedg_prec prec,
                                    iedg_batch* out);
iedg_status iedg_condense_batched(iedg_context ctx, iedg_batch batch, hipStream_t stream);
void iedg_batch_destroy(iedg_batch batch);
/* Tuning of the condensation kernel: width of the register-resident
 * sub-panels of the panel factorisation (8 or 16 columns) for `prec`
 * (IEDG_F64, IEDG_F32 or IEDG_BF16) and elements with n local dofs, kept in
 * the context (thread-safe).  BF16 without an entry of its own uses the
 * FP32 entry.  A width that the register file cannot hold for that case
 * spills to scratch memory (slower, same result).  Untuned: 16 for FP32
 * with n <= 1536 and t <= 512 and for FP64 with n <= 512 and t <= 512,
 * else 8. */
iedg_status iedg_set_leaf_width(iedg_context ctx, iedg_prec prec, int32_t n_local,
                                int32_t leaf_width);
/* Panel width of the condensation's Crout factorisation (section 2.2.1,
 * eq. LS): 64 or 128 columns for FP32 storage (IEDG_F32, IEDG_BF16), 64
 * only for IEDG_F64 (IEDG_ERR_INVALID_ARG otherwise), for elements with n
 * local dofs, kept in the context beside the sub-panel width.  Wider
 * panels read the L and U operands of the Crout updates half as often;
 * narrow elements factor faster in narrow panels.  Untuned: 128 for
 * IEDG_F32 and IEDG_BF16 with n >= 1024, else 64 (BF16 keeps an entry of
 * its own and does not take the FP32 one). */
iedg_status iedg_set_panel_width(iedg_context ctx, iedg_prec prec, int32_t n_local,
                                 int32_t panel_width);

/* ---- a2: assembly of K and R (section 2.2.1, eq. LS) ------------------ */
/* Kbsr = sum_e P_e^T Ke_e P_e in the BSR layout of `mesh` (storage in
 * `prec`, same element type as Ke), R = G + sum_e P_e^T r_e.  Sums over the
 * (at most two) elements sharing a face are taken in ascending element
 * order.  Ke/Kbsr may both be NULL (R only); r, G, R may all be NULL
 * (K only). */
iedg_status iedg_assemble(iedg_context ctx, iedg_mesh mesh, iedg_prec prec,
                          const void* Ke, const double* r, const double* G,
                          void* Kbsr, double* R, hipStream_t stream);

/* ---- a3: BILU(0) (section 2.2.2) -------------------------------------- */
/* Zero-fill block ILU of Kbsr in the mesh's row ordering.  Mbsr has the
 * same layout: lower slots hold L~ (unit block-lower, identity diagonal
 * implied), upper slots hold U~, diagonal slots hold the inverted pivot
 * blocks U~_ii^{-1}.  Mbsr may equal Kbsr (in place).  A singular pivot
 * block latches IEDG_ERR_SINGULAR with the block row. */
iedg_status iedg_factor_ilu0(iedg_context ctx, iedg_mesh mesh, iedg_prec prec,
                             const void* Kbsr, void* Mbsr, hipStream_t stream);

/* Minimum discarded fill ordering of the block rows of K (section 2.2.2,
 * after Persson and Peraire): greedy elimination on the zero-fill pattern;
 * the weight of a row is the squared Frobenius norm of the fill its
 * elimination would drop (blocks A_ik A_kk^{-1} A_kj of pairs (i, j) of live
 * rows coupled to k but not to each other), taken on the matrix as updated
 * by the earlier eliminations (updates kept on the pattern, as BILU(0)
 * makes them); each step eliminates the live row of least weight, ties to
 * the smaller face id.  All in FP64 on the device.  Kbsr: K in the mesh's
 * BSR layout, `prec` storage.  order (host [n_face]) receives the faces in
 * elimination order, to be passed to iedg_mesh_create with ordering 2.
 * A set-up call: it allocates FP64 working arrays (about nnzb + 11 n_face
 * blocks of b x b), synchronises `stream` and frees them before returning.
 * A singular pivot block latches IEDG_ERR_SINGULAR (iedg_sync_status). */
iedg_status iedg_mdf_order(iedg_context ctx, iedg_mesh mesh, iedg_prec prec,
                           const void* Kbsr, int32_t* order, hipStream_t stream);

/* ---- restricted additive Schwarz (section 2.2.2, RAS equation) -------- */
/* M^{-1} = sum_i R_i^0 BILU(0)(K_i)^{-1} R_i^delta over n_sub subdomains,
 * emulated on one GPU.  part (host [n_face]): subdomain of each face (the
 * non-overlapping S_i^0, every subdomain non-empty); S_i^delta adds `delta`
 * layers of faces coupled in K (delta = 0: block Jacobi).  K_i = K on
 * S_i^delta is factored by BILU(0) in the mesh's elimination order
 * restricted to S_i^delta; R_i^0 keeps only the faces of S_i^0 (restricted
 * prolongation: each face takes its own subdomain's value).  All subdomain
 * systems form one block-sparse local system (rows = (subdomain, face)
 * pairs) whose factors Mloc hold nnzb (from iedg_ras_query) blocks of b x b
 * in the factor precision.  Creation allocates the local pattern, maps and
 * two local vectors; factor and apply only launch.  IEDG_ERR_INVALID_ARG for
 * a bad partition. */
typedef struct iedg_ras_s* iedg_ras;
typedef struct {
  int64_t n_sub, delta, n_local_rows, nnzb, n_levels;
} iedg_ras_info;
iedg_status iedg_ras_create(iedg_context ctx, iedg_mesh mesh, int32_t n_sub, const int32_t* part,
                            int32_t delta, iedg_ras* out);
void iedg_ras_destroy(iedg_ras ras);
iedg_status iedg_ras_query(iedg_ras ras, iedg_ras_info* info);
/* Mloc = the BILU(0) factors of every K_i, from K (the mesh's BSR layout,
 * `prec` storage); same factor layout and singular-pivot reporting as
 * iedg_factor_ilu0. */
iedg_status iedg_ras_factor(iedg_context ctx, iedg_ras ras, iedg_prec prec, const void* Kbsr,
                            void* Mloc, hipStream_t stream);
/* y = M^{-1} x (global FP64 vectors [N_t]; y must not alias x). */
iedg_status iedg_ras_apply(iedg_context ctx, iedg_ras ras, iedg_prec prec, const void* Mloc,
                           const double* x, double* y, hipStream_t stream);

/* ---- a4: GMRES (section 2.2.2, eq. LS1) ------------------------------- */
typedef struct {
  int32_t restart;      /* m, Krylov vectors per cycle (>= 1) */
  int32_t max_iters;    /* cap on total Arnoldi steps */
  double rtol;          /* accept when ||R - K x|| / ||R|| <= rtol */
  double inner_factor;  /* inner stop: |g_{j+1}| <= inner_factor*rtol*||M^-1 R|| */
  int32_t precond;      /* 1: M = BILU(0) factors in Mbsr; 0: M = I */
} iedg_gmres_opts;

typedef struct {
  int32_t iters;        /* Arnoldi steps taken */
  int32_t cycles;       /* restart cycles started */
  int32_t converged;    /* 1 when the true residual met rtol */
  double rel_resid;     /* final ||R - K x|| / ||R|| */
} iedg_gmres_info;

/* GMRES workspace of one mesh: the Krylov basis of up to `steps` vectors,
 * reduction partials, the Hessenberg matrix and rotations, device scalars,
 * pinned host slots and two events, all allocated here (steps in [1, 254];
 * IEDG_ERR_INVALID_ARG otherwise, IEDG_ERR_OOM when the allocation fails).
 * A state serves one solve or enqueued cycle at a time; it is not shared
 * between streams. */
typedef struct iedg_gmres_state_s* iedg_gmres_state;
iedg_status iedg_gmres_state_create(iedg_context ctx, iedg_mesh mesh, int32_t steps,
                                    iedg_gmres_state* out);
void iedg_gmres_state_destroy(iedg_gmres_state st);

/* Makes later solves and enqueued cycles of `st` precondition with the RAS
 * `ras` (built on the same mesh): Mbsr is then its factors Mloc.  NULL
 * restores BILU(0) of the whole mesh. */
iedg_status iedg_gmres_state_set_ras(iedg_context ctx, iedg_gmres_state st, iedg_ras ras);

/* Solves M^{-1} K x = M^{-1} R from x0 = 0 (x is output only) by restarted
 * GMRES(opts->restart), restart <= the state's steps (section 2.2.2,
 * eq. LS1).  CGS applied twice per step; Givens rotations; every Krylov
 * quantity FP64.  K (and M) blocks in kprec (mprec) storage.  Uses only the
 * state's workspace (no allocation).  The stopping rule runs on the device:
 * after it fires, the Arnoldi kernels already queued return at once.  The
 * host enqueues steps in chunks of four and, while a chunk is queued,
 * reads the stop flag the previous chunk left (it never waits on the
 * stream inside a cycle); it waits for the stream once per cycle, for the
 * true residual that decides acceptance or restart, so the call returns
 * with the stream synchronised.  Returns IEDG_ERR_NOT_CONVERGED (with *info
 * filled) when max_iters is reached, IEDG_ERR_NONFINITE for a non-finite
 * right-hand side or residual. */
iedg_status iedg_gmres_solve(iedg_context ctx, iedg_mesh mesh, iedg_gmres_state st,
                             iedg_prec kprec, const void* Kbsr, iedg_prec mprec,
                             const void* Mbsr, const double* R, double* x,
                             const iedg_gmres_opts* opts, iedg_gmres_info* info,
                             hipStream_t stream);

/* Capturable GMRES: one cycle of at most `steps` Arnoldi steps from x0 = 0,
 * enqueued with no host synchronisation (it can be captured in a HIP
 * graph).  Every Arnoldi kernel reads a device flag and returns at once
 * after the inner stopping rule has fired, so the cycle stops where
 * iedg_gmres_solve's first cycle would (GMRES(steps) with the same rules).
 * The state owns the Krylov basis and scalars of one mesh; after the stream
 * completes, iedg_gmres_state_read returns iterations, the true relative
 * residual and whether it met rtol (a cycle is not restarted on the
 * device: the caller may fall back to iedg_gmres_solve). */
iedg_status iedg_gmres_enqueue(iedg_context ctx, iedg_mesh mesh, iedg_gmres_state st,
                               iedg_prec kprec, const void* Kbsr, iedg_prec mprec,
                               const void* Mbsr, const double* R, double* x, double rtol,
                               double inner_factor, hipStream_t stream);
/* Synchronous read of the state's results (host). */
iedg_status iedg_gmres_state_read(iedg_context ctx, iedg_gmres_state st, iedg_gmres_info* info);

/* y = K x (kprec blocks, FP64 vectors); exposed for testing and refinement. */
iedg_status iedg_spmv(iedg_context ctx, iedg_mesh mesh, iedg_prec kprec,
                      const void* Kbsr, const double* x, double* y, hipStream_t stream);
/* y = M^{-1} x with BILU(0) factors (forward then backward block sweep). */
iedg_status iedg_ilu0_apply(iedg_context ctx, iedg_mesh mesh, iedg_prec mprec,
                            const void* Mbsr, const double* x, double* y,
                            hipStream_t stream);

/* ---- a5: local back-substitution (section 2.2.1) ---------------------- */
/* z_e = U^{-1} (w_e - U12_e uhat_e) = A_e^{-1} (F_e - B_e uhat_e), where
 * uhat_e gathers the element's t trace dofs from uhat [N_t].  LU, perm,
 * U12 and w as written by iedg_condense (LU, U12 in `prec` storage); w
 * [E][n], uhat, z [E][n] FP64, z in the natural order of A's columns. */
iedg_status iedg_backsolve_local(iedg_context ctx, iedg_mesh mesh, int32_t n_local,
                                 iedg_prec prec, const void* LU, const int32_t* perm,
                                 const void* U12, const double* w, const double* uhat,
                                 double* z, hipStream_t stream);

/* ---- a6: FP64 residual of the uncondensed system ---------------------- */
/* rF_e = F_e - A_e z_e - B_e uhat_e,  rG = G - sum_e P_e^T (C_e z_e + D_e uhat_e),
 * all FP64.  sums (device [4]) receives ||rF||^2, ||rG||^2, ||F||^2,
 * ||G||^2 (deterministic two-stage reductions). */
iedg_status iedg_residual_full(iedg_context ctx, iedg_mesh mesh, int32_t n_local,
                               const double* A, const double* B, const double* C,
                               const double* D, const double* F, const double* G,
                               const double* z, const double* uhat,
                               double* rF, double* rG, double* sums,
                               hipStream_t stream);

/* iedg_residual_full without any library-owned device memory, for callers
 * that cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results
 * (bitwise) as iedg_residual_full; its scratch (q [E][t] and 2E + 2 N_f
 * partial sums) lives in a static device array of 16 MiB (2^21 FP64 values)
 * that each GPU holds from library load to process end; the call allocates
 * nothing and needs E t + 2 E + 2 N_f <= 2^21 (IEDG_ERR_UNSUPPORTED
 * otherwise).  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (different streams, not ordered) race and must not be
 * issued. */
iedg_status iedg_residual_full_noalloc(iedg_context ctx, iedg_mesh mesh, int32_t n_local,
                                       const double* A, const double* B, const double* C,
                                       const double* D, const double* F, const double* G,
                                       const double* z, const double* uhat,
                                       double* rF, double* rG, double* sums,
                                       hipStream_t stream);

/* y += alpha * x over n FP64 values (refinement updates). */
iedg_status iedg_axpy(iedg_context ctx, int64_t n, double alpha, const double* x,
                      double* y, hipStream_t stream);

/* ---- f3: minimal-residual initial guess (section 2.2.1, eq. MinRes2) ---- */
/* The Newton initial guess x0 = sum_j alpha_j x_j over s previous solutions
 * x_j = (z_j, uhat_j), with alpha minimising ||R(x0)||^2 (both blocks of
 * the residual), found by Levenberg-Marquardt with finite-difference
 * gradients.  R is the residual of the uncondensed Newton system plus a
 * componentwise cubic term (eps = 0: the linear residual of a6):
 *   R_NS,e = F_e - A_e z_e - B_e uhat_e - eps z_e^3,
 *   R_FL   = G - sum_e P_e^T (C_e z_e + D_e uhat_e) - eps uhat^3.
 * Each evaluation pass reads the FP64 element blocks once for a batch of up
 * to s_max + 1 points (a trial and its s finite-difference neighbours).
 * Layouts: Zprev [s][E][n] and Uprev [s][N_t] FP64 device (previous
 * solution j at index j, most recent first); A, B, C, D, F, G as for
 * iedg_residual_full.
 * iedg_mr_create allocates the state (two sets of s_max + 1 residual
 * vectors of E n + N_t values, per-point partial sums, the Gram matrix and
 * a pinned readback area); 1 <= s_max <= 8 (IEDG_ERR_UNSUPPORTED
 * otherwise); the points of a pass must fit in LDS: (s + 1)(n + t) FP64
 * values <= 160 KiB.
 * iedg_mr_residual: R [m][E n + N_t] (device, element rows e-major then the
 * trace) and sums [m] (device, ||R_k||^2) at the m <= s_max + 1 points
 * point_k = sum_j beta[k s + j] x_j (beta host, [m][s]).  Launches only.
 * iedg_mr_guess: alpha [s] (host), z0 [E][n] and u0 [N_t] (device) = the
 * combination; synchronises `stream` after each pass and each Gram matrix
 * (the s x s damped normal equations are solved on the host).  Algorithm
 * (opts may be NULL: max_iters 20, lambda0 1e-3, fd_step 1e-7, tol 1e-10,
 * ftol 1e-10):
 * start at alpha = e_1 and lambda0; Jacobian columns by forward differences
 * with steps fd_step max(1, |alpha_i|); step (J^T J + lambda diag(J^T J)) d
 * = -J^T r; accept if the objective decreases (lambda /= 10, floor 1e-12),
 * else lambda *= 10 (at most 10 tries per step); stop after max_iters
 * accepted steps, when no try is accepted, when max|d| <= tol (1 +
 * max|alpha|), when an accepted step lowers the objective by no more than
 * ftol of its value, or at a zero objective.  info: accepted steps, passes, the
 * objective at e_1 and at alpha. */
typedef struct iedg_mr_s* iedg_mr;
typedef struct {
  int32_t max_iters;
  double lambda0, fd_step, tol, ftol;
} iedg_mr_opts;
typedef struct {
  int32_t iters, passes;
  double obj0, obj;
} iedg_mr_info;
iedg_status iedg_mr_create(iedg_context ctx, iedg_mesh mesh, int32_t n_local, int32_t s_max,
                           iedg_mr* out);
void iedg_mr_destroy(iedg_mr mr);
iedg_status iedg_mr_residual(iedg_context ctx, iedg_mr mr, const double* A, const double* B,
                             const double* C, const double* D, const double* F, const double* G,
                             double eps, int32_t s, const double* Zprev, const double* Uprev,
                             int32_t m, const double* beta, double* R, double* sums,
                             hipStream_t stream);
iedg_status iedg_mr_guess(iedg_context ctx, iedg_mr mr, const double* A, const double* B,
                          const double* C, const double* D, const double* F, const double* G,
                          double eps, int32_t s, const double* Zprev, const double* Uprev,
                          const iedg_mr_opts* opts, double* alpha, double* z0, double* u0,
                          iedg_mr_info* info, hipStream_t stream);

/* ---- measured device ceilings (the roofline report's second denominator) */
/* An MFMA loop: n_wg workgroups of 512 threads, each wave issuing `iters`
 * rounds of 8 independent 16x16 accumulations with the instruction the
 * condensation issues for `prec` (IEDG_F64: FP64 16x16x4; IEDG_F32: FP32
 * 16x16x4; IEDG_BF16: BF16 16x16x16 with FP32 accumulation) on operands of
 * one.  sink (device, n_wg * 512 doubles) receives each thread's sum of its
 * accumulators (8 chains of 4 entries), 32 K iters with K = 4 (FP64, FP32)
 * or 16 (BF16), which checks that the loop ran; *flops (host) = 2 16 16 K 8 8 iters n_wg, the
 * floating-point operations of the launch.  1 <= iters <= 2^20.
 * Asynchronous on `stream` (time it with events on that stream). */
iedg_status iedg_probe_mfma(iedg_context ctx, iedg_prec prec, int32_t n_wg,
                            int32_t iters, double* sink, double* flops,
                            hipStream_t stream);
/* STREAM triad a = b + s c over n FP64 values (device arrays, n even and
 * positive, 16-byte aligned; IEDG_ERR_INVALID_ARG otherwise): 24 n bytes of
 * HBM traffic.  Asynchronous on `stream`. */
iedg_status iedg_probe_triad(iedg_context ctx, int64_t n, const double* b,
                             const double* c, double s, double* a,
                             hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* IEDG_H */
