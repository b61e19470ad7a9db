"""GPU tests of the serving form: every request meets the tolerance, a
request's result is bitwise the same served alone and in a concurrent mix
(with evictions and re-admissions), and it agrees with the FP64 oracle."""
import sys

import numpy as np
import pytest
import torch

import oracle
from synth import SEED_BASE
from synth.matrices import MeshCase

from helpers import host_case
from gpu_util import rel

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


SEED = SEED_BASE + 4
CASES = [MeshCase(0, (2, 2, 1), 1), MeshCase(1, (2, 1, 1), 2), MeshCase(2, (1, 1, 2), 1),
         MeshCase(3, (1, 2, 1), 2), MeshCase(4, (1, 1, 1), 1), MeshCase(5, (2, 2, 2), 1),
         MeshCase(6, (2, 1, 1), 3), MeshCase(7, (1, 2, 1), 4)]


def _serve(ctx, requests, n_slots, budget, progress=None):
    from paper_1605_01020_amd.serve import Server
    srv = Server(ctx, CASES, SEED, budget_bytes=budget, n_slots=n_slots, keep_results=True)
    done = srv.run(requests, real_time=False, progress=progress, every=5)
    stats = dict(srv.stats)
    srv.close()
    return {(r.sim, r.rhs): r for r in done}, stats


def test_serving_mix_invariance(ctx):
    from paper_1605_01020_amd.serve import poisson_requests
    from paper_1605_01020_amd.batch import Simulation
    reqs = poisson_requests(SEED, 24, 100.0, len(CASES))
    big = 10 * sum(Simulation.footprint(c) for c in CASES)
    _say("serving alone (1 slot, everything resident)")
    alone, st_alone = _serve(ctx, [r for r in poisson_requests(SEED, 24, 100.0, len(CASES))], 1, big)
    assert st_alone["evictions"] == 0
    _say("serving mixed (4 slots, budget forcing evictions)")
    # room for the largest simulation and a fifth of it: admitting the p = 4
    # simulation evicts the others, and the p = 3 one cannot stay beside it
    tight = 1.2 * max(Simulation.footprint(c) for c in CASES)
    calls = []
    mixed, st_mix = _serve(ctx, reqs, 4, tight, progress=lambda k, n: calls.append((k, n)))
    assert calls == [(k, 24) for k in range(5, 25, 5)]  # every 5 completions
    assert st_mix["evictions"] > 0 and st_mix["misses"] > st_alone["misses"]
    assert set(alone) == set(mixed) and len(alone) == 24
    for key, a in alone.items():
        b = mixed[key]
        assert a.rho <= 1e-8 and b.rho <= 1e-8, (key, a.rho, b.rho)
        assert torch.equal(a.uhat, b.uhat), key
        assert torch.equal(a.z, b.z), key
    # latency bookkeeping
    for r in mixed.values():
        assert r.done >= r.start >= 0


def test_serving_result_matches_oracle(ctx):
    from paper_1605_01020_amd.serve import Request
    from paper_1605_01020_amd.batch import Simulation
    big = 10 * sum(Simulation.footprint(c) for c in CASES)
    reqs = [Request(0, 1, 3, 0.0), Request(1, 5, 2, 0.0), Request(2, 1, 4, 0.0), Request(3, 6, 1, 0.0),
            Request(4, 7, 2, 0.0)]
    got, st = _serve(ctx, reqs, 2, big)
    assert st["hits"] == 1 and st["misses"] == 4
    for (sid, rhs), r in got.items():
        c = CASES[sid]
        _say(f"oracle for sim {sid} rhs {rhs}")
        m, spec, blocks, G = host_case(c.dims, c.p, seed=SEED, mesh_id=c.mesh_id, rhs=rhs)
        tm = oracle.TraceMesh(m.elem_faces(), m.n_face, spec.b)
        ref = oracle.newton_step_solve(tm, blocks, G, restart=100, rtol=1e-13)
        assert rel(r.uhat.cpu().numpy(), ref["uhat"]) <= 1e-7
        assert rel(r.z.cpu().numpy(), np.stack(ref["z"])) <= 1e-7
