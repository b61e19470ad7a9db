"""Restricted additive Schwarz (RAS) preconditioner with delta-level overlap
and BILU(0) subdomain solves (section 2.2.2, RAS equation).

Parity: pinned (tests): N = 1 reduces to BILU(0) of K; delta = 0 is block
Jacobi, equal to BILU(0) of K with the couplings between subdomains
removed; on small meshes the operator equals a dense construction from
selection matrices and a scalar ILU(0) of each dense subdomain matrix.

Given a partition of the faces (the entities of the trace system) into N
non-overlapping subdomains S_i^0, the delta-level overlap subdomain S_i^delta
adds delta layers of the face-to-face coupling graph (faces coupled in K).
K_i is K restricted to S_i^delta, factored by BILU(0) under the given order
restricted to S_i^delta, and

    M^{-1} x = sum_i R_i^0 BILU(0)(K_i)^{-1} R_i^delta x,

where R_i^delta takes the entries of x on S_i^delta and R_i^0 returns only
the entries of the local solution that belong to S_i^0 (restricted
prolongation: every face takes its value from its own subdomain).
"""
import numpy as np

from .bilu0 import bilu0, bilu0_apply


class _SubMesh:
    """The pattern of K restricted to a face subset (global face ids)."""

    def __init__(self, tmesh, faces):
        keep = np.zeros(tmesh.n_face, dtype=bool)
        keep[faces] = True
        self.n_face, self.b, self.n_trace = tmesh.n_face, tmesh.b, tmesh.n_trace
        self.pattern = [[g for g in tmesh.pattern[f] if keep[g]] if keep[f] else [] for f in range(tmesh.n_face)]


def overlap(tmesh, owned, delta):
    """S^delta: owned faces plus delta layers of coupled faces (sorted ids)."""
    cur = set(int(f) for f in owned)
    for _ in range(delta):
        cur |= {g for f in cur for g in tmesh.pattern[f]}
    return np.array(sorted(cur), dtype=np.int64)


def ras_setup(tmesh, K, part, delta, order):
    """Subdomain factors.  part: subdomain of every face; order: a global
    face order whose restriction to each S_i^delta is its elimination order."""
    part = np.asarray(part)
    subs = []
    for i in range(int(part.max()) + 1):
        owned = np.nonzero(part == i)[0]
        Sd = overlap(tmesh, owned, delta)
        sm = _SubMesh(tmesh, Sd)
        inS = np.zeros(tmesh.n_face, dtype=bool)
        inS[Sd] = True
        order_i = np.array([f for f in order if inS[f]], dtype=np.int64)
        Ki = {(f, g): K[(f, g)] for f in Sd for g in sm.pattern[f]}
        subs.append({"owned": owned, "faces": Sd, "mesh": sm, "fac": bilu0(sm, Ki, order_i)})
    return subs


def ras_apply(tmesh, subs, x):
    b = tmesh.b
    y = np.zeros(tmesh.n_trace)
    for s in subs:
        xi = np.zeros(tmesh.n_trace)
        dofs = (s["faces"][:, None] * b + np.arange(b)[None, :]).ravel()
        xi[dofs] = x[dofs]                                   # R_i^delta
        zi = bilu0_apply(s["mesh"], s["fac"], xi)            # BILU(0)(K_i)^{-1}
        own = (s["owned"][:, None] * b + np.arange(b)[None, :]).ravel()
        y[own] = zi[own]                                     # R_i^0
    return y
