"""GPU parity of the minimum discarded fill ordering (iedg_mdf_order) against
the oracle's MDF: the same K (the oracle's, uploaded into the library's BSR
layout) gives the same order; BILU(0) factors and the GMRES solve under that
order match the oracle's under the same order."""
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle.assembly import matvec
from synth import StructuredHexMesh

from helpers import host_case
from gpu_util import dev, host_blocks_to_dev, bsr_from_oracle, oracle_from_bsr, rel

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


def _random_K(tm, seed, diag=6.0, scale=0.5):
    rng = np.random.default_rng(seed)
    K = {}
    for f in range(tm.n_face):
        for g in tm.pattern[f]:
            K[(f, g)] = rng.standard_normal((tm.b, tm.b)) * scale + (diag * np.eye(tm.b) if f == g else 0)
    return K


@pytest.mark.parametrize("dims,b,ordering", [((4, 4, 4), 45, "colour"), ((3, 2, 2), 20, "natural"),
                                             ((2, 2, 1), 125, "colour")])
def test_mdf_order_equals_oracle_random_blocks(ctx, dims, b, ordering):
    """Random blocks on the face pattern (the 4x4x4 case has the p = 2
    subdomain shape of the smallest workload; b = 125 is the p = 4 face)."""
    _say(f"mdf random K dims={dims} b={b}")
    m = StructuredHexMesh(*dims)
    tm = oracle.TraceMesh(m.elem_faces(), m.n_face, b)
    K = _random_K(tm, sum(dims) + b)
    mesh = api.Mesh(ctx, m.elem_faces(), m.n_face, b, ordering=ordering)
    q = mesh.query()
    got = api.mdf_order(ctx, mesh, dev(bsr_from_oracle(mesh, K, q)))
    ctx.sync_status()
    ref = oracle.mdf_order(tm, K)
    assert np.array_equal(got, ref)
    # FP32 storage: the order of the rounded matrix
    K32 = {key: blk.astype(np.float32).astype(np.float64) for key, blk in K.items()}
    got32 = api.mdf_order(ctx, mesh, dev(bsr_from_oracle(mesh, K32, q).astype(np.float32)), prec=1)
    assert np.array_equal(got32, oracle.mdf_order(tm, K32))


@pytest.mark.parametrize("dims,p", [((2, 2, 2), 1), ((3, 2, 1), 2)])
def test_mdf_solve_matches_oracle(ctx, dims, p):
    """Condensed K of a seeded mesh: MDF order equal to the oracle's; BILU(0)
    under it equal to the oracle's (<= 1e-11); GMRES takes the oracle's
    iteration count and reaches the same solution."""
    _say(f"mdf solve dims={dims} p={p}")
    m, spec, blocks, G = host_case(dims, p)
    tm = oracle.TraceMesh(m.elem_faces(), m.n_face, spec.b)
    Ks, rs = oracle.condense_all(blocks)
    K, R = oracle.assemble(tm, Ks, rs, G)
    ref_order = oracle.mdf_order(tm, K)
    mesh0 = api.Mesh(ctx, m.elem_faces(), m.n_face, spec.b)
    order = api.mdf_order(ctx, mesh0, dev(bsr_from_oracle(mesh0, K, mesh0.query())))
    assert np.array_equal(order, ref_order)
    mesh = api.Mesh(ctx, m.elem_faces(), m.n_face, spec.b, ordering="given", order=order)
    qm = mesh.query()
    assert np.array_equal(qm["order"], order)
    # the GPU pipeline under the MDF order
    d = host_blocks_to_dev(blocks)
    fac = api.condense(ctx, d["A"], d["B"], d["C"], d["D"], d["F"])
    Kd, Rd = api.assemble(ctx, mesh, Ke=fac["Ke"], r=fac["r"], G=dev(G))
    Md = api.factor_ilu0(ctx, mesh, Kd)
    ctx.sync_status()
    ofac = oracle.bilu0(tm, K, order)
    got = oracle_from_bsr(mesh, Md.cpu().numpy(), qm)
    scale = max(np.abs(v).max() for v in K.values())
    for key, Lb in ofac["L"].items():
        assert np.abs(got[key] - Lb).max() <= 1e-11 * scale
    for key, Ub in ofac["U"].items():
        if key[0] != key[1]:
            assert np.abs(got[key] - Ub).max() <= 1e-11 * scale
    for i, Ui in ofac["Uinv"].items():
        assert np.abs(got[(i, i)] - Ui).max() <= 1e-11 * np.abs(Ui).max()
    x, info = api.gmres_solve(ctx, mesh, Kd, Md, Rd, restart=50, rtol=1e-10)
    u_ref, oinfo = oracle.gmres(lambda v: matvec(tm, K, v), lambda v: oracle.bilu0_apply(tm, ofac, v), R, 50, 1e-10)
    assert info["converged"] and info["iters"] == oinfo["iters"]
    assert rel(x.cpu().numpy(), u_ref) <= 5e-10
    # the level count of the MDF order is the oracle's
    assert mesh.n_levels == oracle.level_sets(tm, order).max() + 1
