"""ctypes binding of the device-side input generator (libsynth.so).

Writes the same seeded element blocks as synth.matrices straight into
device memory (torch CUDA tensors), so large workloads never pass through
host memory.  Values agree with the host generator bit for bit (the same
Philox words, and the same series for ln, cos and sin evaluated in the same
order).
"""
import ctypes
import os

import numpy as np

from .matrices import (ElementSpec, MAT_A, MAT_B, MAT_C, MAT_D, MAT_F, MAT_G,
                       G_STREAM, dist_params, make_tag)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        L.synth_gen_matrix.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                       ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_void_p]
        L.synth_gen_matrix.restype = ctypes.c_int
        L.synth_philox.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_uint64,
                                   ctypes.c_void_p]
        L.synth_philox.restype = ctypes.c_int
        _lib = L
    return _lib


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _gen(out, rows, cols, n_stream, stream0, tag, seed, diag, sigma):
    # chunk over streams (grid.y is limited)
    per = 60000
    for s0 in range(0, n_stream, per):
        cnt = min(per, n_stream - s0)
        ptr = out.data_ptr() + s0 * rows * cols * 8
        rc = lib().synth_gen_matrix(ctypes.c_void_p(ptr), rows, cols, cnt, (stream0 + s0) & 0xFFFFFFFF,
                                    tag, seed, diag, sigma, _stream())
        if rc != 0:
            raise RuntimeError(f"synth_gen_matrix failed ({rc})")


def gen_blocks(spec, seed, mesh_id, n_elem, which="ABCD", rhs=0, elem0=0, out=None):
    """Device tensors for element blocks of elements elem0 .. elem0+n_elem-1."""
    import torch
    n, t = spec.n, spec.t
    shapes = {"A": (MAT_A, n, n), "B": (MAT_B, n, t), "C": (MAT_C, t, n),
              "D": (MAT_D, t, t), "F": (MAT_F, n, 1)}
    res = {} if out is None else out
    for key in which:
        mat, r, c = shapes[key]
        if key not in res:
            res[key] = torch.empty((n_elem, r, c) if key != "F" else (n_elem, r),
                                   dtype=torch.float64, device="cuda")
        diag, sigma = dist_params(spec, mat)
        _gen(res[key], r, c, n_elem, elem0, make_tag(mesh_id, mat, rhs if key == "F" else 0),
             seed, diag, sigma)
    return res


def gen_trace_rhs(spec, seed, mesh_id, n_face, rhs=0, out=None, count=None):
    """G on the device: n_face * b values, or the first `count` of the same
    stream (the trace size of another numbering)."""
    import torch
    total = n_face * spec.b if count is None else int(count)
    if out is None:
        out = torch.empty(total, dtype=torch.float64, device="cuda")
    diag, sigma = dist_params(spec, MAT_G)
    _gen(out, 1, total, 1, G_STREAM, make_tag(mesh_id, MAT_G, rhs), seed, diag, sigma)
    return out


def philox_words(counters, seed):
    """Raw Philox4x32-10 words on the device for an int array [count, 4]."""
    import torch
    ctr = torch.as_tensor(np.ascontiguousarray(counters, dtype=np.uint32).view(np.int32), device="cuda")
    out = torch.empty_like(ctr)
    rc = lib().synth_philox(ctypes.c_void_p(out.data_ptr()), ctr.shape[0], ctypes.c_void_p(ctr.data_ptr()),
                            seed, _stream())
    if rc != 0:
        raise RuntimeError("synth_philox failed")
    return out.cpu().numpy().view(np.uint32)
