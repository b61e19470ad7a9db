"""Pins for the oracle's restricted additive Schwarz preconditioner, each
independent of oracle/ras.py's bookkeeping: N = 1 is BILU(0) of K; delta = 0
is block Jacobi (BILU(0) of K without the couplings between subdomains);
and a dense construction from 0/1 selection matrices, overlaps from powers
of the face adjacency matrix, and a scalar ILU(0) of each dense subdomain
matrix."""
import numpy as np
import pytest

import oracle
from synth import StructuredHexMesh

from test_oracle import _point_ilu0_product


def _setup(dims, b, seed):
    m = StructuredHexMesh(*dims)
    tm = oracle.TraceMesh(m.elem_faces(), m.n_face, b)
    rng = np.random.default_rng(seed)
    K = {}
    for f in range(tm.n_face):
        for g in tm.pattern[f]:
            K[(f, g)] = rng.standard_normal((b, b)) * 0.4 + (5.0 * np.eye(b) if f == g else 0)
    return m, tm, K


def test_face_slabs_partition():
    m = StructuredHexMesh(4, 2, 3)
    for n in (1, 2, 4):
        part = m.face_slabs(n)
        assert part.min() == 0 and part.max() == n - 1
        # every face belongs to the slab of one of its elements
        ef = m.elem_faces()
        slab = (np.arange(m.n_elem) // (m.ny * m.nz)) * n // m.nx
        for f in range(m.n_face):
            assert part[f] in {int(slab[e]) for e in range(m.n_elem) if f in ef[e]}


def test_ras_single_subdomain_is_bilu0():
    m, tm, K = _setup((3, 2, 2), 3, 1)
    order = oracle.greedy_colour_order(tm)
    part = np.zeros(tm.n_face, dtype=np.int64)
    x = np.random.default_rng(2).standard_normal(tm.n_trace)
    fac = oracle.bilu0(tm, K, order)
    for delta in (0, 1):
        subs = oracle.ras_setup(tm, K, part, delta, order)
        assert np.abs(oracle.ras_apply(tm, subs, x) - oracle.bilu0_apply(tm, fac, x)).max() <= 1e-15 * np.abs(x).max()


class _Pattern:
    def __init__(self, tm, keep):
        self.n_face, self.b, self.n_trace = tm.n_face, tm.b, tm.n_trace
        self.pattern = [[g for g in tm.pattern[f] if keep(f, g)] for f in range(tm.n_face)]


def test_ras_delta0_is_block_jacobi():
    m, tm, K = _setup((4, 2, 2), 3, 3)
    part = m.face_slabs(2)
    order = oracle.natural_order(tm)
    bj = _Pattern(tm, lambda f, g: part[f] == part[g])
    Kbj = {(f, g): K[(f, g)] for f in range(tm.n_face) for g in bj.pattern[f]}
    fac = oracle.bilu0(bj, Kbj, order)
    x = np.random.default_rng(4).standard_normal(tm.n_trace)
    subs = oracle.ras_setup(tm, K, part, 0, order)
    assert np.abs(oracle.ras_apply(tm, subs, x) - oracle.bilu0_apply(bj, fac, x)).max() <= 1e-13 * np.abs(x).max()


@pytest.mark.parametrize("delta", [0, 1, 2])
@pytest.mark.parametrize("ordering", ["natural", "colour"])
def test_ras_equals_dense_construction(delta, ordering):
    m, tm, K = _setup((3, 2, 1), 2, 5 + delta)
    b, nf = tm.b, tm.n_face
    part = m.face_slabs(3)
    order = oracle.natural_order(tm) if ordering == "natural" else oracle.greedy_colour_order(tm)
    Kd = np.zeros((tm.n_trace, tm.n_trace))
    for (f, g), blk in K.items():
        Kd[f * b:(f + 1) * b, g * b:(g + 1) * b] = blk
    adj = np.zeros((nf, nf), dtype=np.int64)
    for f in range(nf):
        for g in tm.pattern[f]:
            adj[f, g] = 1
    reach = np.linalg.matrix_power(np.eye(nf, dtype=np.int64) + adj, delta) > 0
    pos = np.empty(nf, dtype=np.int64)
    pos[order] = np.arange(nf)
    x = np.random.default_rng(9).standard_normal(tm.n_trace)
    y = np.zeros(tm.n_trace)
    subs = oracle.ras_setup(tm, K, part, delta, order)
    for i in range(part.max() + 1):
        owned = part == i
        Sd = np.nonzero(reach[owned].any(axis=0))[0]
        assert np.array_equal(Sd, subs[i]["faces"])
        Sd = Sd[np.argsort(pos[Sd])]                     # elimination order
        dofs = (Sd[:, None] * b + np.arange(b)[None, :]).ravel()
        Rd = np.zeros((len(dofs), tm.n_trace))
        Rd[np.arange(len(dofs)), dofs] = 1.0             # R_i^delta
        Ki = Rd @ Kd @ Rd.T
        mask = np.kron(adj[np.ix_(Sd, Sd)] > 0, np.ones((b, b), dtype=bool))
        Mi = _point_ilu0_product(Ki, mask)
        R0 = Rd * np.repeat(owned[Sd], b)[:, None]       # R_i^0: owned rows only
        y += R0.T @ np.linalg.solve(Mi, Rd @ x)
    got = oracle.ras_apply(tm, subs, x)
    assert np.abs(got - y).max() <= 1e-12 * np.abs(y).max()
