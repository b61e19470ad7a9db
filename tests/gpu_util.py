"""Helpers for the GPU parity tests (host <-> device layout conversions)."""
import numpy as np
import torch


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def stack(blocks, key):
    return np.stack([b[key] for b in blocks])


def host_blocks_to_dev(blocks):
    return {k: dev(stack(blocks, k)) for k in "ABCDF"}


def bsr_from_oracle(mesh, K, q):
    """Oracle dict {(f, g): block} -> array in the library's BSR slot layout
    (column-major blocks, i.e. the transpose of each row-major block)."""
    order, row_ptr, col_face = q["order"], q["row_ptr"], q["col_face"]
    out = np.empty((len(col_face), mesh.b, mesh.b))
    for i, f in enumerate(order):
        for s in range(row_ptr[i], row_ptr[i + 1]):
            out[s] = K[(int(f), int(col_face[s]))].T
    return out


def oracle_from_bsr(mesh, arr, q):
    order, row_ptr, col_face = q["order"], q["row_ptr"], q["col_face"]
    out = {}
    for i, f in enumerate(order):
        for s in range(row_ptr[i], row_ptr[i + 1]):
            out[(int(f), int(col_face[s]))] = np.asarray(arr[s]).T
    return out


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
