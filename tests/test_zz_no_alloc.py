"""The allocation-free residual entry point (iedg_residual_full_noalloc),
called through the C ABI, against iedg_residual_full: bitwise equal outputs
on two calls in a row, the second on a smaller mesh (the shared static
scratch keeps the first call's contents), and the size limit rejected
before anything is enqueued."""
import ctypes
import sys

import numpy as np
import pytest
import torch

from helpers import host_case
from gpu_util import host_blocks_to_dev, dev

pytestmark = pytest.mark.gpu
api = pytest.importorskip("paper_1605_01020_amd.api")


def _say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def _case(ctx, dims, p):
    m, spec, blocks, G = host_case(dims, p, rhs=1)
    mesh = api.Mesh(ctx, m.elem_faces(), m.n_face, spec.b)
    d = host_blocks_to_dev(blocks)
    rng = np.random.default_rng(sum(dims) + p)
    z = dev(rng.standard_normal((m.n_elem, spec.n)))
    u = dev(rng.standard_normal(m.n_face * spec.b))
    return mesh, spec, d, dev(G), z, u


def _call(ctx, fn, mesh, spec, d, G, z, u):
    E = mesh.n_elem
    rF = torch.full((E, spec.n), float("nan"), dtype=torch.float64, device="cuda")
    rG = torch.full_like(G, float("nan"))
    sums = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    s0 = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = fn(ctx.h, mesh.h, spec.n, p(d["A"]), p(d["B"]), p(d["C"]), p(d["D"]), p(d["F"]), p(G), p(z), p(u),
            p(rF), p(rG), p(sums), s0)
    ctx.check(st)
    return rF, rG, sums


def test_noalloc_residual_equals_residual_full():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = api.Context()
    L = ctx.L
    for dims, p in [((2, 2, 2), 2), ((2, 1, 1), 1)]:   # the second call is smaller
        _say(f"noalloc residual dims={dims} p={p}")
        mesh, spec, d, G, z, u = _case(ctx, dims, p)
        ref = _call(ctx, L.iedg_residual_full, mesh, spec, d, G, z, u)
        got = _call(ctx, L.iedg_residual_full_noalloc, mesh, spec, d, G, z, u)
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            assert torch.equal(a, b), dims
        assert torch.isfinite(got[2]).all() and got[2][2] > 0
    ctx.sync_status()


def test_noalloc_residual_rejects_oversize():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from synth import StructuredHexMesh
    ctx = api.Context()
    # E t + 2 E + 2 N_f > 2^21: 24 x 24 x 8 elements of p = 3 (t = 480)
    hm = StructuredHexMesh(24, 24, 8)
    mesh = api.Mesh(ctx, hm.elem_faces(), hm.n_face, 80)
    assert hm.n_elem * 480 + 2 * hm.n_elem + 2 * hm.n_face > 2 ** 21
    x = torch.zeros(16, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(x.data_ptr())
    s0 = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = ctx.L.iedg_residual_full_noalloc(ctx.h, mesh.h, 1280, p, p, p, p, p, p, p, p, p, p, p, s0)
    assert st == -7
    assert b"static" in ctx.L.iedg_last_error(ctx.h)
