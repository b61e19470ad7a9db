"""Pins for the minimum discarded fill ordering of the oracle.

Each check is independent of oracle/mdf.py's block formulas: a chain
pattern whose exact LU has no fill, and a dense brute force that eliminates
one face at a time from a dense copy of the matrix, masks the result to the
block pattern, and takes the candidate whose dropped entries have the least
squared Frobenius norm."""
import numpy as np
import pytest

import oracle
from oracle.mdf import mdf_order
from synth import StructuredHexMesh


class _Chain:
    """Block-tridiagonal pattern: face f couples to f-1, f, f+1."""

    def __init__(self, n_face, b):
        self.n_face, self.b, self.n_trace = n_face, b, n_face * b
        self.pattern = [[g for g in (f - 1, f, f + 1) if 0 <= g < n_face] for f in range(n_face)]


def _random_K(tm, rng, diag=6.0, scale=0.5):
    b = tm.b
    K = {}
    for f in range(tm.n_face):
        for g in tm.pattern[f]:
            K[(f, g)] = rng.standard_normal((b, b)) * scale + (diag * np.eye(b) if f == g else 0)
    return K


def test_mdf_chain_is_natural_and_discards_nothing():
    ch = _Chain(10, 3)
    K = _random_K(ch, np.random.default_rng(2))
    rec = {}
    order = mdf_order(ch, K, record=rec)
    assert list(order) == list(range(ch.n_face))
    # the chosen face discards nothing at every step (an end of the chain)
    for cand, w, k in zip(rec["candidates"], rec["weights"], order):
        assert w[list(cand).index(k)] == 0.0
    # interior faces of the initial chain would discard fill (i-1, i+1)
    assert (rec["weights"][0][1:-1] > 0).all()


def _brute_force_steps(tm, K, order):
    """Replay `order` on a dense copy; at each step return the dense weights
    of every live candidate (ascending face id)."""
    b, nf = tm.b, tm.n_face
    N = nf * b
    R = np.zeros((N, N))
    mask = np.zeros((N, N), dtype=bool)
    for (f, g), blk in K.items():
        R[f * b:(f + 1) * b, g * b:(g + 1) * b] = blk
        mask[f * b:(f + 1) * b, g * b:(g + 1) * b] = True
    live = np.ones(nf, dtype=bool)
    steps = []
    for k in order:
        rows_live = np.repeat(live, b)
        ws = []
        for c in np.nonzero(live)[0]:
            cs = slice(c * b, (c + 1) * b)
            keep = rows_live.copy()
            keep[cs] = False
            S = R[:, cs] @ np.linalg.solve(R[cs, cs], R[cs, :])
            S[~keep, :] = 0.0
            S[:, ~keep] = 0.0
            ws.append(float(np.sum(S[~mask] ** 2)))
        steps.append((np.nonzero(live)[0], np.array(ws)))
        ks = slice(k * b, (k + 1) * b)
        keep = rows_live.copy()
        keep[ks] = False
        S = R[:, ks] @ np.linalg.solve(R[ks, ks], R[ks, :])
        upd = np.outer(keep, keep) & mask
        R[upd] -= S[upd]
        live[k] = False
    return steps


@pytest.mark.parametrize("dims,b,seed", [((2, 2, 2), 2, 5), ((3, 2, 1), 3, 9)])
def test_mdf_choices_equal_dense_brute_force(dims, b, seed):
    mesh = StructuredHexMesh(*dims)
    tm = oracle.TraceMesh(mesh.elem_faces(), mesh.n_face, b)
    K = _random_K(tm, np.random.default_rng(seed))
    rec = {}
    order = mdf_order(tm, K, record=rec)
    assert sorted(order) == list(range(tm.n_face))
    steps = _brute_force_steps(tm, K, order)
    for s, ((cand, wd), k) in enumerate(zip(steps, order)):
        assert list(cand) == list(rec["candidates"][s])
        wo = rec["weights"][s]
        assert np.allclose(wo, wd, rtol=1e-10, atol=1e-12 * max(1.0, wd.max()))
        # the dense minimum, ties to the smaller face id
        assert cand[int(np.argmin(wd))] == k
    # a non-trivial order: not the natural one
    assert list(order) != list(range(tm.n_face))


def test_mdf_pivots_are_the_bilu0_pivots_of_its_order():
    """The elimination MDF performs is BILU(0) in right-looking form: the
    pivot block met when a face is chosen is its U~_kk under that order."""
    mesh = StructuredHexMesh(2, 2, 2)
    tm = oracle.TraceMesh(mesh.elem_faces(), mesh.n_face, 3)
    K = _random_K(tm, np.random.default_rng(4))
    rec = {}
    order = mdf_order(tm, K, record=rec)
    fac = oracle.bilu0(tm, K, order)
    for k, P in rec["pivot"].items():
        assert np.abs(P - fac["U"][(k, k)]).max() <= 1e-12 * np.abs(P).max()
