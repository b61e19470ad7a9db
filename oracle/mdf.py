"""Minimum discarded fill (MDF) ordering for BILU(0) (section 2.2.2, which
applies the MDF reordering of Persson and Peraire 2008 at subdomain level).

Parity: pinned (tests): on block-tridiagonal matrices MDF discards nothing
and returns the natural order; on small meshes every greedy choice equals
the brute-force minimum computed from a dense copy of the partially
eliminated matrix; the pivot blocks met during the ordering equal the
BILU(0) pivot blocks of the resulting order.

Greedy elimination on the zero-fill pattern of K.  Eliminating block row k
next would add  -A_ik A_kk^{-1} A_kj  to every pair (i, j) of not yet
eliminated faces coupled to k.  Pairs inside the pattern receive the update
(exactly what BILU(0) does); pairs outside it are dropped.  The weight of k
is the squared Frobenius norm of what would be dropped:

    w_k = sum over live i != j in pattern(k), (i, j) not in pattern, of
          || A_ik A_kk^{-1} A_kj ||_F^2

At every step the live face of least weight is eliminated (ties go to the
smaller face id), the remaining matrix is updated on the pattern, and the
weights of its live neighbours are recomputed.  Readings: the weights are
taken on the partially eliminated matrix (the updates are kept), in FP64.
"""
import numpy as np


def _weight(tmesh, A, pattern_set, k, live):
    nb = [g for g in tmesh.pattern[k] if g != k and live[g]]
    X = {j: np.linalg.solve(A[(k, k)], A[(k, j)]) for j in nb}
    s = 0.0
    for i in nb:
        for j in nb:
            if i != j and (i, j) not in pattern_set:
                fill = A[(i, k)] @ X[j]
                s += float(np.sum(fill * fill))
    return s


def mdf_order(tmesh, K, record=None):
    """Greedy MDF order of the faces of K ({(f, g): b x b block}).  With
    `record` (a dict), also returns each step's weights and pivot blocks."""
    A = {key: np.array(blk, dtype=np.float64, copy=True) for key, blk in K.items()}
    pattern_set = set(K.keys())
    nf = tmesh.n_face
    live = np.ones(nf, dtype=bool)
    w = np.array([_weight(tmesh, A, pattern_set, k, live) for k in range(nf)])
    order = []
    for _ in range(nf):
        cand = np.nonzero(live)[0]
        k = int(cand[np.argmin(w[cand])])  # first minimum: smallest id among ties
        if record is not None:
            record.setdefault("weights", []).append(w[cand].copy())
            record.setdefault("candidates", []).append(cand.copy())
            record.setdefault("pivot", {})[k] = A[(k, k)].copy()
        order.append(k)
        live[k] = False
        nb = [g for g in tmesh.pattern[k] if g != k and live[g]]
        for i in nb:
            Lik = np.linalg.solve(A[(k, k)].T, A[(i, k)].T).T  # A_ik A_kk^{-1}
            for j in nb:
                if (i, j) in pattern_set:
                    A[(i, j)] = A[(i, j)] - Lik @ A[(k, j)]
        for g in nb:
            w[g] = _weight(tmesh, A, pattern_set, g, live)
    return np.asarray(order, dtype=np.int64)
