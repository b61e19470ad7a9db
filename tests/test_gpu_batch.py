"""GPU tests of the batched form: the device-driven GMRES cycle against the
host-driven one, the persistent batched condensation against the
one-launch-per-mesh condensation, the whole batch against the FP64 oracle,
and graph replays against the eager run."""
import sys

import numpy as np
import pytest
import torch

import oracle
from synth import SEED_BASE
from synth.matrices import MeshCase, Workload

from helpers import host_case
from gpu_util import host_blocks_to_dev, dev, rel

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


SEED = SEED_BASE + 3
# degrees 1 to 4: the batched condensation instantiations for n <= 512,
# n <= 1536 (p = 3, b = 80) and n <= 2560 (p = 4, b = 125), and the sweep
# lane groups of every face size, all run here
CASES = [MeshCase(0, (2, 2, 1), 1), MeshCase(1, (2, 1, 1), 2), MeshCase(2, (1, 1, 2), 1),
         MeshCase(3, (1, 2, 1), 2), MeshCase(4, (1, 1, 1), 1), MeshCase(5, (2, 1, 1), 3),
         MeshCase(6, (1, 2, 1), 4)]


def _trace_system(ctx, dims, p, prec=0):
    m, spec, blocks, G = host_case(dims, p)
    mesh = api.Mesh(ctx, m.elem_faces(), m.n_face, spec.b)
    d = host_blocks_to_dev(blocks)
    fac = api.condense(ctx, d["A"], d["B"], d["C"], d["D"], d["F"], prec=prec)
    K, R = api.assemble(ctx, mesh, Ke=fac["Ke"], r=fac["r"], G=dev(G), prec=prec)
    M = api.factor_ilu0(ctx, mesh, K, prec=prec)
    return mesh, K, M, R


@pytest.mark.parametrize("dims,p", [((2, 2, 2), 1), ((2, 2, 1), 3), ((2, 1, 1), 4)])
@pytest.mark.parametrize("prec", [0, 1])
def test_gmres_enqueue_equals_host_cycle(ctx, prec, dims, p):
    _say(f"gmres_enqueue vs gmres_solve prec={prec} dims={dims} p={p}")
    mesh, K, M, R = _trace_system(ctx, dims, p, prec)
    x_h, info_h = api.gmres_solve(ctx, mesh, K, M, R, restart=50, rtol=1e-10, kprec=prec, mprec=prec)
    assert info_h["cycles"] == 1 and info_h["converged"]
    st = api.GmresState(ctx, mesh, 50)
    x_d = torch.full_like(R, float("nan"))
    st.enqueue(K, M, R, x_d, 1e-10, kprec=prec, mprec=prec)
    torch.cuda.synchronize()
    info_d = st.read()
    assert torch.equal(x_d, x_h)
    assert info_d["iters"] == info_h["iters"] and info_d["converged"]
    assert info_d["rel_resid"] == info_h["rel_resid"]
    # a cycle cut at `steps` stops where the host solve with max_iters = steps stops
    st2 = api.GmresState(ctx, mesh, 2)
    st2.enqueue(K, M, R, x_d, 1e-12, kprec=prec, mprec=prec)
    x_h2, info_h2 = api.gmres_solve(ctx, mesh, K, M, R, restart=2, rtol=1e-12, max_iters=2, kprec=prec,
                                    mprec=prec, raise_on_fail=False)
    torch.cuda.synchronize()
    info_d2 = st2.read()
    assert info_d2["iters"] == 2 and not info_d2["converged"]
    assert torch.equal(x_d, x_h2) and info_d2["rel_resid"] == info_h2["rel_resid"]
    # zero right-hand side: x = 0 and nothing iterates
    Z = torch.zeros_like(R)
    st.enqueue(K, M, Z, x_d, 1e-10, kprec=prec, mprec=prec)
    torch.cuda.synchronize()
    info_z = st.read()
    assert info_z["iters"] == 0 and info_z["converged"] and not x_d.any()
    st.close()
    st2.close()


def test_batched_condense_equals_single_launch(ctx):
    """One persistent launch over meshes of four element sizes computes what
    one launch per mesh computes, bitwise; a second run (the queue counter
    reset on the stream) again; a segment without elements is skipped."""
    from paper_1605_01020_amd.batch import Simulation
    from paper_1605_01020_amd import F32
    _say("batched condensation vs per-mesh condensation")
    sims = [Simulation(ctx, c, SEED) for c in CASES]
    for s in sims:
        s.generate()
    # a non-default sub-panel width for p = 2: the plan takes the context's
    # width per size, as iedg_condense does
    n_p2 = next(s.n for s in sims if s.case.p == 2)
    api.set_leaf_width(ctx, n_p2, 8, prec=F32)
    try:
        empty = {k: v[:0] for k, v in sims[0].inp.items() if v is not None}
        empty_out = {k: v[:0] for k, v in sims[0].fac.items()}
        pl = api.CondenseBatch(ctx, [s.condense_segment() for s in sims] + [(empty, empty_out)], prec=sims[0].prec)
        assert len(pl.sizes) == 4
        refs = []
        for s in sims:
            i = s.inp
            refs.append(api.condense(ctx, i["A"], i["B"], i["C"], i["D"], i["F"], prec=s.prec))
        for rep in range(2):
            for s in sims:
                for k in ("Ke", "r", "LU"):
                    s.fac[k].fill_(float("nan"))
            pl.run()
            torch.cuda.synchronize()
            ctx.sync_status()
            for s, ref in zip(sims, refs):
                for k in ("LU", "perm", "U12", "L21", "Ke", "w", "r"):
                    assert torch.equal(ref[k], s.fac[k]), (rep, s.case, k)
        pl.close()
    finally:
        api.set_leaf_width(ctx, n_p2, 16, prec=F32)
    for s in sims:
        s.close()


def _oracle_solution(case):
    m, spec, blocks, G = host_case(case.dims, case.p, seed=SEED, mesh_id=case.mesh_id)
    tm = oracle.TraceMesh(m.elem_faces(), m.n_face, spec.b)
    res = oracle.newton_step_solve(tm, blocks, G, restart=100, rtol=1e-13)
    return res["uhat"], np.stack(res["z"])


def test_batch_group_matches_oracle_and_graph_replays(ctx):
    from paper_1605_01020_amd.batch import Simulation, BatchGroup
    _say("batch group eager + graph")
    sims = [Simulation(ctx, c, SEED, tol=1e-8) for c in CASES]
    for s in sims:
        s.generate()
    grp = BatchGroup(ctx, sims)
    grp.enqueue()
    res = grp.finish()
    snap = [(s.uhat.clone(), s.z.clone(), s.sums.clone()) for s in sims]
    for s, r in zip(sims, res):
        assert r.converged, (s.case, r)
        assert r.eager_steps == 0, (s.case, r.rho_hist)
        u_ref, z_ref = _oracle_solution(s.case)
        assert rel(s.uhat.cpu().numpy(), u_ref) <= 1e-7, s.case
        assert rel(s.z.cpu().numpy(), z_ref) <= 1e-7, s.case
    grp.capture()
    for rep in range(3):
        # eager work and clobbered outputs between replays
        for s in sims:
            s.uhat.fill_(float("nan"))
            s.z.fill_(float("nan"))
            api.spmv(ctx, s.mesh, s.K, s.R, prec=s.prec, y=s.Rc)
        torch.cuda.synchronize()
        grp.run()
        torch.cuda.synchronize()
        for s, (u, z, sm) in zip(sims, snap):
            assert torch.equal(s.uhat, u), (rep, s.case)
            assert torch.equal(s.z, z), (rep, s.case)
            assert torch.equal(s.sums, sm), (rep, s.case)
    ctx.sync_status()
    grp.close()
    for s in sims:
        s.close()


def test_run_batch_groups_under_budget(ctx):
    from paper_1605_01020_amd.batch import run_batch, Simulation
    _say("run_batch with a small memory budget")
    wl = Workload("small_batch", SEED, CASES, restart=100, rtol=1e-8)
    # the largest (p = 4) mesh and a fifth of it: not every mesh fits beside it
    budget = max(Simulation.footprint(c) for c in CASES) * 1.2
    assert budget < sum(Simulation.footprint(c) for c in CASES)
    out = run_batch(ctx, wl, budget_bytes=budget, replays=2)
    assert out["groups"] >= 2
    assert [r.mesh_id for r in out["results"]] == [c.mesh_id for c in CASES]
    assert all(r.converged for r in out["results"])
