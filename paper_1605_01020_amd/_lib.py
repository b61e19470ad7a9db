"""ctypes declarations of the C ABI in include/iedg.h (libiedg.so)."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libiedg.so")

c_int32, c_int64, c_double, c_void_p = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
P = c_void_p

F64, F32, BF16 = 0, 1, 2
STATUS = {0: "ok", -1: "invalid argument", -2: "singular pivot", -3: "not converged",
          -4: "non-finite value", -5: "out of device memory", -6: "HIP runtime error",
          -7: "unsupported"}


class MeshInfo(ctypes.Structure):
    _fields_ = [("n_elem", c_int64), ("n_face", c_int64), ("face_dofs", c_int64),
                ("n_trace", c_int64), ("nnzb", c_int64), ("n_levels", c_int64)]


class GmresOpts(ctypes.Structure):
    _fields_ = [("restart", c_int32), ("max_iters", c_int32), ("rtol", c_double),
                ("inner_factor", c_double), ("precond", c_int32)]


class GmresInfo(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("cycles", c_int32), ("converged", c_int32),
                ("rel_resid", c_double)]


class RasInfo(ctypes.Structure):
    _fields_ = [("n_sub", c_int64), ("delta", c_int64), ("n_local_rows", c_int64), ("nnzb", c_int64),
                ("n_levels", c_int64)]


class MrOpts(ctypes.Structure):
    _fields_ = [("max_iters", c_int32), ("lambda0", ctypes.c_double), ("fd_step", ctypes.c_double),
                ("tol", ctypes.c_double), ("ftol", ctypes.c_double)]


class MrInfo(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("passes", c_int32), ("obj0", ctypes.c_double), ("obj", ctypes.c_double)]


class CondenseSegment(ctypes.Structure):
    _fields_ = [("n_elem", c_int32), ("A", P), ("B", P), ("C", P), ("D", P), ("F", P),
                ("LU", P), ("perm", P), ("U12", P), ("L21", P), ("w", P), ("Ke", P), ("r", P)]


# name -> (restype, argtypes)
SIGNATURES = {
    "iedg_create": (c_int32, [ctypes.POINTER(c_void_p), ctypes.c_int]),
    "iedg_destroy": (None, [P]),
    "iedg_last_error": (ctypes.c_char_p, [P]),
    "iedg_status_string": (ctypes.c_char_p, [c_int32]),
    "iedg_sync_status": (c_int32, [P, P, ctypes.POINTER(c_int64)]),
    "iedg_mesh_create": (c_int32, [P, c_int32, c_int32, c_int32, P, c_int32, P, ctypes.POINTER(c_void_p)]),
    "iedg_mesh_create_slots": (c_int32, [P, c_int32, c_int32, c_int32, c_int32, P, c_int32, P,
                                         ctypes.POINTER(c_void_p)]),
    "iedg_mesh_destroy": (None, [P]),
    "iedg_mesh_query": (c_int32, [P, ctypes.POINTER(MeshInfo), P, P, P, P]),
    "iedg_condense": (c_int32, [P, c_int32, c_int32, c_int32, c_int32, P, P, P, P, P,
                                P, P, P, P, P, P, P, P]),
    "iedg_batch_create": (c_int32, [P, c_int32, ctypes.POINTER(CondenseSegment), c_int32, c_int32,
                                    c_int32, ctypes.POINTER(c_void_p)]),
    "iedg_batch_create_sized": (c_int32, [P, c_int32, ctypes.POINTER(CondenseSegment), P, P,
                                          c_int32, ctypes.POINTER(c_void_p)]),
    "iedg_condense_batched": (c_int32, [P, P, P]),
    "iedg_mr_create": (c_int32, [P, P, c_int32, c_int32, ctypes.POINTER(c_void_p)]),
    "iedg_mr_destroy": (None, [P]),
    "iedg_mr_residual": (c_int32, [P, P, P, P, P, P, P, P, ctypes.c_double, c_int32, P, P, c_int32, P, P, P, P]),
    "iedg_mr_guess": (c_int32, [P, P, P, P, P, P, P, P, ctypes.c_double, c_int32, P, P, ctypes.POINTER(MrOpts), P,
                                P, P, ctypes.POINTER(MrInfo), P]),
    "iedg_batch_destroy": (None, [P]),
    "iedg_set_leaf_width": (c_int32, [P, c_int32, c_int32, c_int32]),
    "iedg_set_panel_width": (c_int32, [P, c_int32, c_int32, c_int32]),
    "iedg_condense_rhs": (c_int32, [P, c_int32, c_int32, c_int32, c_int32, P, P, P, P, P, P, P]),
    "iedg_assemble": (c_int32, [P, P, c_int32, P, P, P, P, P, P]),
    "iedg_factor_ilu0": (c_int32, [P, P, c_int32, P, P, P]),
    "iedg_mdf_order": (c_int32, [P, P, c_int32, P, P, P]),
    "iedg_ras_create": (c_int32, [P, P, c_int32, P, c_int32, ctypes.POINTER(c_void_p)]),
    "iedg_ras_destroy": (None, [P]),
    "iedg_ras_query": (c_int32, [P, ctypes.POINTER(RasInfo)]),
    "iedg_ras_factor": (c_int32, [P, P, c_int32, P, P, P]),
    "iedg_ras_apply": (c_int32, [P, P, c_int32, P, P, P, P]),
    "iedg_gmres_state_set_ras": (c_int32, [P, P, P]),
    "iedg_gmres_solve": (c_int32, [P, P, P, c_int32, P, c_int32, P, P, P, ctypes.POINTER(GmresOpts),
                                   ctypes.POINTER(GmresInfo), P]),
    "iedg_gmres_state_create": (c_int32, [P, P, c_int32, ctypes.POINTER(c_void_p)]),
    "iedg_gmres_enqueue": (c_int32, [P, P, P, c_int32, P, c_int32, P, P, P, c_double, c_double, P]),
    "iedg_gmres_state_read": (c_int32, [P, P, ctypes.POINTER(GmresInfo)]),
    "iedg_gmres_state_destroy": (None, [P]),
    "iedg_spmv": (c_int32, [P, P, c_int32, P, P, P, P]),
    "iedg_ilu0_apply": (c_int32, [P, P, c_int32, P, P, P, P]),
    "iedg_backsolve_local": (c_int32, [P, P, c_int32, c_int32, P, P, P, P, P, P, P]),
    "iedg_residual_full": (c_int32, [P, P, c_int32, P, P, P, P, P, P, P, P, P, P, P, P]),
    "iedg_residual_full_noalloc": (c_int32, [P, P, c_int32, P, P, P, P, P, P, P, P, P, P, P, P]),
    "iedg_axpy": (c_int32, [P, c_int64, c_double, P, P, P]),
    "iedg_probe_mfma": (c_int32, [P, c_int32, c_int32, c_int32, P, ctypes.POINTER(c_double), P]),
    "iedg_probe_triad": (c_int32, [P, c_int64, P, P, c_double, P, P]),
}

_lib = None


def load(path=LIB_PATH):
    """Load libiedg.so; raises if it is missing (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: the HIP library is required "
                           "(run __graft_entry__.build())")
    L = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def exported_symbols():
    return list(SIGNATURES)
