"""GPU parity of the restricted additive Schwarz preconditioner (iedg_ras_*)
against the oracle's RAS: the operator on random vectors, GMRES iteration
counts and solutions; one subdomain is bitwise BILU(0) of the whole mesh."""
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle.assembly import matvec

from helpers import host_case
from gpu_util import dev, host_blocks_to_dev, bsr_from_oracle, rel

pytestmark = pytest.mark.gpu
api = pytest.importorskip("paper_1605_01020_amd.api")


def _say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = api.Context()
    yield c
    torch.cuda.synchronize()


@pytest.fixture(autouse=True)
def _clean_status(request):
    if "ctx" in request.fixturenames:
        request.getfixturevalue("ctx").clear_status()
    yield


@pytest.fixture(scope="module")
def system():
    m, spec, blocks, G = host_case((6, 2, 2), 1)
    tm = oracle.TraceMesh(m.elem_faces(), m.n_face, spec.b)
    Ks, rs = oracle.condense_all(blocks)
    K, R = oracle.assemble(tm, Ks, rs, G)
    return m, spec, tm, K, R


@pytest.mark.parametrize("ordering", ["colour", "natural"])
@pytest.mark.parametrize("n_sub,delta", [(2, 0), (2, 1), (3, 1), (6, 0), (6, 2)])
def test_ras_apply_matches_oracle(ctx, system, n_sub, delta, ordering):
    m, spec, tm, K, R = system
    _say(f"ras apply N={n_sub} delta={delta} {ordering}")
    mesh = api.Mesh(ctx, m.elem_faces(), m.n_face, spec.b, ordering=ordering)
    q = mesh.query()
    part = m.face_slabs(n_sub)
    ras = api.Ras(ctx, mesh, part, delta)
    Kd = dev(bsr_from_oracle(mesh, K, q))
    Ml = ras.factor(Kd)
    ctx.sync_status()
    subs = oracle.ras_setup(tm, K, part, delta, q["order"])
    assert ras.n_local_rows == sum(len(s["faces"]) for s in subs)
    x = np.random.default_rng(n_sub + 10 * delta).standard_normal(tm.n_trace)
    y = ras.apply(Ml, dev(x)).cpu().numpy()
    assert rel(y, oracle.ras_apply(tm, subs, x)) <= 1e-12
    ras.close()


def test_ras_one_subdomain_is_bilu0_bitwise(ctx, system):
    m, spec, tm, K, R = system
    mesh = api.Mesh(ctx, m.elem_faces(), m.n_face, spec.b)
    Kd = dev(bsr_from_oracle(mesh, K, mesh.query()))
    M = api.factor_ilu0(ctx, mesh, Kd)
    x = dev(np.random.default_rng(1).standard_normal(tm.n_trace))
    y0 = api.ilu0_apply(ctx, mesh, M, x)
    for delta in (0, 1):
        ras = api.Ras(ctx, mesh, np.zeros(m.n_face, np.int32), delta)
        Ml = ras.factor(Kd)
        assert torch.equal(Ml, M)
        assert torch.equal(ras.apply(Ml, x), y0)
        ras.close()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n_sub,delta", [(3, 0), (3, 1)])
def test_ras_gmres_matches_oracle(ctx, system, n_sub, delta, prec):
    m, spec, tm, K, R = system
    _say(f"ras gmres N={n_sub} delta={delta} prec={prec}")
    mesh = api.Mesh(ctx, m.elem_faces(), m.n_face, spec.b)
    q = mesh.query()
    part = m.face_slabs(n_sub)
    ras = api.Ras(ctx, mesh, part, delta)
    Kbsr = bsr_from_oracle(mesh, K, q)
    Kd = dev(Kbsr if prec == 0 else Kbsr.astype(np.float32))
    Ml = ras.factor(Kd, prec=prec)
    st = api.GmresState(ctx, mesh, 50)
    st.set_ras(ras)
    x, info = api.gmres_solve(ctx, mesh, Kd, Ml, dev(R), 50, 1e-10, kprec=prec, mprec=prec, state=st)
    ctx.sync_status()
    Kref = K if prec == 0 else {k: v.astype(np.float32).astype(np.float64) for k, v in K.items()}
    subs = oracle.ras_setup(tm, Kref, part, delta, q["order"])
    u, oinfo = oracle.gmres(lambda v: matvec(tm, Kref, v), lambda v: oracle.ras_apply(tm, subs, v), R, 50, 1e-10)
    assert info["converged"]
    if prec == 0:
        assert info["iters"] == oinfo["iters"]
        assert rel(x.cpu().numpy(), u) <= 5e-10
    else:
        # FP32 factors applied in FP32 arithmetic: the count may differ by one
        assert abs(info["iters"] - oinfo["iters"]) <= 1
        assert rel(x.cpu().numpy(), u) <= 1e-8
    # the device-driven cycle with the same preconditioner reaches the same iterate
    x2 = torch.full_like(x, float("nan"))
    st.enqueue(Kd, Ml, dev(R), x2, 1e-10, kprec=prec, mprec=prec)
    torch.cuda.synchronize()
    assert torch.equal(x2, x) and st.read()["iters"] == info["iters"]
    st.close()
    ras.close()


def test_ras_rejects_bad_partition(ctx, system):
    m, spec, tm, K, R = system
    mesh = api.Mesh(ctx, m.elem_faces(), m.n_face, spec.b)
    part = m.face_slabs(2)
    part[0] = 5   # subdomains 2..4 empty
    with pytest.raises(api.IedgError):
        api.Ras(ctx, mesh, part, 1)
