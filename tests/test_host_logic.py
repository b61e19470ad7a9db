"""Host-side logic of the batched and serving forms (no GPU)."""
import numpy as np
import pytest

from synth.matrices import workload, MeshCase


def test_plan_groups_packs_every_mesh_once_under_budget():
    from paper_1605_01020_amd.batch import plan_groups, Simulation
    wl = workload(3)
    budget = 200e9
    groups = plan_groups(wl.meshes, budget)
    ids = sorted(c.mesh_id for g in groups for c in g)
    assert ids == list(range(len(wl.meshes)))
    for g in groups:
        assert sum(Simulation.footprint(c) for c in g) <= budget
    with pytest.raises(ValueError):
        plan_groups(wl.meshes, 1e9)


def test_nnzb_estimate_matches_structure_table():
    # nonzero face blocks of K for the meshes of the batched configuration
    from paper_1605_01020_amd.batch import _nnzb_estimate
    from synth.mesh import StructuredHexMesh
    for dims, nnzb in (((4, 4, 4), 2160), ((16, 16, 8), 68096), ((6, 6, 6), 7236), ((8, 8, 4), 8576),
                       ((12, 12, 6), 28800)):
        assert _nnzb_estimate(StructuredHexMesh(*dims)) == nnzb


def test_poisson_requests_are_seeded_and_poisson():
    from paper_1605_01020_amd.serve import poisson_requests
    a = poisson_requests(7, 4000, 50.0, 64)
    b = poisson_requests(7, 4000, 50.0, 64)
    assert [(r.sim, r.rhs, r.arrival) for r in a] == [(r.sim, r.rhs, r.arrival) for r in b]
    gaps = np.diff([r.arrival for r in a])
    assert abs(gaps.mean() - 1 / 50.0) < 0.1 / 50.0          # exponential mean 1/rate
    assert abs(gaps.std() - 1 / 50.0) < 0.1 / 50.0            # and std 1/rate
    sims = np.array([r.sim for r in a])
    assert sims.min() == 0 and sims.max() == 63
    # right-hand side ids count per simulation from 1
    seen = {}
    for r in a:
        seen[r.sim] = seen.get(r.sim, 0) + 1
        assert r.rhs == seen[r.sim]
