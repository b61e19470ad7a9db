"""Pins for the FP64 oracle: every check here is independent of the oracle's
own formulas (dense direct solves, determinant identities, the defining
property of ILU(0), Krylov invariants, validity of orderings)."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from oracle.assembly import to_dense, matvec
from oracle.bilu0 import product_blocks
from oracle.ordering import greedy_colours
from synth import StructuredHexMesh, ElementSpec, element_inputs, SEED_BASE

from helpers import host_case, dense_uncondensed

TINY = [((1, 1, 1), 1), ((2, 2, 2), 1), ((2, 2, 1), 2)]


def _tmesh(mesh, spec):
    return oracle.TraceMesh(mesh.elem_faces(), mesh.n_face, spec.b)


@pytest.mark.parametrize("dims,p", TINY)
def test_solve_matches_dense_uncondensed(dims, p):
    mesh, spec, blocks, G = host_case(dims, p)
    tm = _tmesh(mesh, spec)
    res = oracle.newton_step_solve(tm, blocks, G, restart=50, rtol=1e-13)
    M, rhs = dense_uncondensed(tm, blocks, G)
    sol = np.linalg.solve(M, rhs)
    mine = np.concatenate([np.concatenate(res["z"]), res["uhat"]])
    assert np.linalg.norm(sol - mine) <= 1e-11 * np.linalg.norm(sol)
    # the assembled K and R are the exact Schur complement of the dense system
    E, n = tm.n_elem, spec.n
    S = M[E * n:, E * n:] - M[E * n:, :E * n] @ np.linalg.solve(M[:E * n, :E * n], M[:E * n, E * n:])
    assert np.abs(to_dense(tm, res["K"]) - S).max() <= 1e-13 * np.abs(S).max()
    Rd = rhs[E * n:] - M[E * n:, :E * n] @ np.linalg.solve(M[:E * n, :E * n], rhs[:E * n])
    assert np.abs(res["R"] - Rd).max() <= 1e-13 * np.abs(Rd).max()
    # the oracle's own residual agrees with the dense residual
    r_dense = np.linalg.norm(rhs - M @ mine) / np.linalg.norm(rhs)
    assert abs(res["info"]["rho_full"] - r_dense) <= 1e-15 + 1e-6 * r_dense


def test_schur_determinant_identity():
    spec = ElementSpec(1)
    blk = element_inputs(spec, SEED_BASE, 0, 3)
    Ke, re, _ = oracle.condense_element(blk["A"], blk["B"], blk["C"], blk["D"], blk["F"])
    M = np.block([[blk["A"], blk["B"]], [blk["C"], blk["D"]]])
    sM, lM = np.linalg.slogdet(M)
    sA, lA = np.linalg.slogdet(blk["A"])
    sK, lK = np.linalg.slogdet(Ke)
    assert sM == sA * sK
    assert abs(lM - (lA + lK)) <= 1e-10 * abs(lM)


def test_condensed_rhs_reproduces_bordered_solve():
    spec = ElementSpec(1)
    blk = element_inputs(spec, SEED_BASE, 0, 4)
    g = np.random.default_rng(0).standard_normal(spec.t)
    M = np.block([[blk["A"], blk["B"]], [blk["C"], blk["D"]]])
    sol = np.linalg.solve(M, np.concatenate([blk["F"], g]))
    Ke, re, _ = oracle.condense_element(blk["A"], blk["B"], blk["C"], blk["D"], blk["F"])
    y = np.linalg.solve(Ke, g + re)
    assert np.linalg.norm(y - sol[spec.n:]) <= 1e-13 * np.linalg.norm(sol)
    z = oracle.backsolve_element(blk["A"], blk["B"], blk["F"], y)
    assert np.linalg.norm(z - sol[:spec.n]) <= 1e-13 * np.linalg.norm(sol)
    # first block row of the Newton system holds to rounding
    assert np.linalg.norm(blk["F"] - blk["A"] @ z - blk["B"] @ y) <= 1e-13 * np.linalg.norm(blk["F"])


def test_bilu0_reproduces_K_on_pattern():
    mesh, spec, blocks, G = host_case((2, 2, 2), 1)
    tm = _tmesh(mesh, spec)
    Ks, rs = oracle.condense_all(blocks)
    K, R = oracle.assemble(tm, Ks, rs, G)
    for order in (oracle.natural_order(tm), oracle.greedy_colour_order(tm)):
        fac = oracle.bilu0(tm, K, order)
        prod = product_blocks(tm, fac)
        scale = max(np.abs(blk).max() for blk in K.values())
        err = max(np.abs(prod[key] - K[key]).max() for key in K)
        assert err <= 1e-13 * scale
        # some product blocks fall outside the pattern: the discarded fill
        assert any(key not in K for key in prod)
        # the stored pivot inverses are inverses
        for i, Ui in fac["Uinv"].items():
            assert np.abs(Ui @ fac["U"][(i, i)] - np.eye(tm.b)).max() <= 1e-13


class _Chain:
    """A block-tridiagonal pattern: face f couples to f-1, f, f+1."""

    def __init__(self, n_face, b):
        self.n_face, self.b, self.n_trace = n_face, b, n_face * b
        self.pattern = [[g for g in (f - 1, f, f + 1) if 0 <= g < n_face] for f in range(n_face)]


def test_bilu0_exact_on_block_tridiagonal():
    rng = np.random.default_rng(7)
    ch = _Chain(9, 4)
    K = {}
    for f in range(ch.n_face):
        for g in ch.pattern[f]:
            K[(f, g)] = rng.standard_normal((4, 4)) * 0.3 + (4.0 * np.eye(4) if f == g else 0)
    fac = oracle.bilu0(ch, K, np.arange(ch.n_face))
    prod = product_blocks(ch, fac)
    assert set(prod) == set(K)  # no fill at all
    for key in K:
        assert np.abs(prod[key] - K[key]).max() <= 1e-14 * 4
    Kd = to_dense(ch, K)
    x = rng.standard_normal(ch.n_trace)
    assert np.linalg.norm(oracle.bilu0_apply(ch, fac, Kd @ x) - x) <= 1e-13 * np.linalg.norm(x)


def test_single_element_mesh_ilu_is_exact():
    mesh, spec, blocks, G = host_case((1, 1, 1), 1)
    tm = _tmesh(mesh, spec)
    res = oracle.newton_step_solve(tm, blocks, G, restart=10, rtol=1e-12)
    assert res["info"]["iters"] == 1
    Kd = to_dense(tm, res["K"])
    sol = np.linalg.solve(Kd, res["R"])
    assert np.linalg.norm(res["uhat"] - sol) <= 1e-13 * np.linalg.norm(sol)


def _random_system(N, seed):
    rng = np.random.default_rng(seed)
    Kd = np.eye(N) * 3 + rng.standard_normal((N, N)) / np.sqrt(N)
    return Kd, rng.standard_normal(N)


def test_gmres_krylov_invariants():
    mesh, spec, blocks, G = host_case((2, 2, 2), 1)
    tm = _tmesh(mesh, spec)
    Ks, rs = oracle.condense_all(blocks)
    K, R = oracle.assemble(tm, Ks, rs, G)
    fac = oracle.bilu0(tm, K, oracle.greedy_colour_order(tm))
    Kmv = lambda v: matvec(tm, K, v)
    Minv = lambda v: oracle.bilu0_apply(tm, fac, v)
    x, info = oracle.gmres(Kmv, Minv, R, restart=30, rtol=1e-12, record=True)
    V = info["V"][0]
    k = V.shape[0] - 1
    assert np.abs(V @ V.T - np.eye(k + 1)).max() <= 1e-13
    Hbar = np.zeros((k + 1, k))
    for j, col in enumerate(info["H_raw"][:k]):
        Hbar[:j + 2, j] = col
    AV = np.stack([Minv(Kmv(V[j])) for j in range(k)], axis=1)
    assert np.abs(AV - V.T @ Hbar).max() <= 1e-12 * np.abs(AV).max()
    est = np.array(info["est_hist"])
    assert (np.diff(est) <= 1e-15 * est[0]).all()
    Kd = to_dense(tm, K)
    assert np.linalg.norm(x - np.linalg.solve(Kd, R)) <= 1e-11 * np.linalg.norm(x)


def test_gmres_finite_termination_unpreconditioned():
    N = 40
    Kd, R = _random_system(N, 3)
    x, info = oracle.gmres(lambda v: Kd @ v, lambda v: v.copy(), R, restart=N, rtol=1e-12)
    assert info["converged"] and info["iters"] <= N and info["cycles"] == 1
    assert np.linalg.norm(R - Kd @ x) <= 1e-12 * np.linalg.norm(R)


def test_gmres_restarted_residual_non_increasing():
    N = 60
    Kd, R = _random_system(N, 5)
    x, info = oracle.gmres(lambda v: Kd @ v, lambda v: v.copy(), R, restart=4, rtol=1e-10)
    hist = np.array(info["true_hist"])
    assert info["converged"] and info["cycles"] > 2
    assert (np.diff(hist) <= 1e-14).all()
    assert np.linalg.norm(x - np.linalg.solve(Kd, R)) <= 1e-9 * np.linalg.norm(x)


def test_gmres_not_converged_reported():
    N = 60
    Kd, R = _random_system(N, 5)
    x, info = oracle.gmres(lambda v: Kd @ v, lambda v: v.copy(), R, restart=2, rtol=1e-14, max_cycles=2)
    assert not info["converged"] and info["rel_resid"] > 1e-14


@pytest.mark.parametrize("dims", [(2, 2, 2), (3, 2, 4), (4, 4, 4)])
def test_colour_order_is_valid(dims):
    mesh = StructuredHexMesh(*dims)
    tm = oracle.TraceMesh(mesh.elem_faces(), mesh.n_face, 1)
    col = greedy_colours(tm)
    assert col.max() + 1 == 6
    for f in range(tm.n_face):
        assert all(col[g] != col[f] for g in tm.pattern[f] if g != f)
    for order in (oracle.natural_order(tm), oracle.greedy_colour_order(tm)):
        lev = oracle.level_sets(tm, order)
        pos = np.empty(tm.n_face, dtype=np.int64)
        pos[order] = np.arange(tm.n_face)
        for f in range(tm.n_face):
            lower = [lev[g] for g in tm.pattern[f] if pos[g] < pos[f]]
            assert lev[f] == (max(lower) + 1 if lower else 0)
            # a level is an independent set
            assert all(lev[g] != lev[f] for g in tm.pattern[f] if g != f)
    lev_c = oracle.level_sets(tm, oracle.greedy_colour_order(tm))
    assert lev_c.max() + 1 == 6


def _point_ilu0_product(dense, mask):
    """Scalar zero-fill ILU(0) (IKJ form, no pivoting) of a dense matrix on
    the point pattern `mask`, written from the textbook definition; returns
    the product L U of its unit-lower and upper factors."""
    a = dense.copy()
    N = a.shape[0]
    for i in range(1, N):
        for k in np.nonzero(mask[i, :i])[0]:
            a[i, k] /= a[k, k]
            cols = np.nonzero(mask[i, k + 1:])[0] + k + 1
            a[i, cols] -= a[i, k] * a[k, cols]
    L = np.tril(a, -1) + np.eye(N)
    U = np.triu(a)
    return L @ U


@pytest.mark.parametrize("ordering", ["natural", "colour"])
def test_point_ilu0_equals_block_ilu0(ordering):
    """With face-private trace dofs every nonzero block of K is dense, so the
    scalar ILU(0) on K's point pattern and the b x b block ILU(0) define the
    same preconditioner M = L U (the block form only groups the arithmetic).
    Random blocks on the face pattern of a 3x2x2 mesh, b = 3, diagonally
    dominant pivot blocks (the scalar form does not pivot)."""
    mesh = StructuredHexMesh(3, 2, 2)
    b = 3
    tm = oracle.TraceMesh(mesh.elem_faces(), mesh.n_face, b)
    rng = np.random.default_rng(11)
    K = {}
    for f in range(tm.n_face):
        for g in tm.pattern[f]:
            K[(f, g)] = rng.standard_normal((b, b)) * 0.2 + (6.0 * np.eye(b) if f == g else 0)
    order = oracle.natural_order(tm) if ordering == "natural" else oracle.greedy_colour_order(tm)
    fac = oracle.bilu0(tm, K, order)
    # dense copies in the elimination order: point index = position * b + l
    pos = fac["pos"]
    N = tm.n_trace
    dense = np.zeros((N, N))
    mask = np.zeros((N, N), dtype=bool)
    for (f, g), blk in K.items():
        r, c = pos[f] * b, pos[g] * b
        dense[r:r + b, c:c + b] = blk
        mask[r:r + b, c:c + b] = True
    Mp = _point_ilu0_product(dense, mask)
    Mb = np.zeros((N, N))
    for (f, g), blk in product_blocks(tm, fac).items():
        r, c = pos[f] * b, pos[g] * b
        Mb[r:r + b, c:c + b] = blk
    assert np.abs(Mp - Mb).max() <= 1e-13 * np.abs(dense).max()
    # not trivially K: both discard the same fill outside the pattern
    assert np.abs(Mp - dense)[~mask].max() > 1e-3
    assert np.abs(Mp - dense)[mask].max() <= 1e-13 * np.abs(dense).max()
