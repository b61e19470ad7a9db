"""Assembly of the trace system K dU = R (section 2.2.1, eq. LS).

Parity: pinned through the dense uncondensed solve (tests: the assembled K
and R equal the Schur complement of the dense system), and the closed-form
block count nnzb = N_f + 30 E of a structured hex mesh.  ``to_dense`` and
``matvec`` are pinned with it (the dense comparison goes through
``to_dense``; GMRES on ``matvec`` reproduces the dense solve).

K is returned as a dict {(f, g): b x b block}; every element adds the
blocks of K_e of each pair of its local slots (36 face pairs in the
face-private numbering) to the block of the units they map to, in slot
order.  R = G + sum_e P_e^T r_e, where P_e^T adds every local dof into its
global dof (several local dofs of one element may share a global dof in the
IEDG numbering).
"""
import numpy as np


def assemble(tmesh, Ks, rs, G):
    b = tmesh.b
    K = {}
    for e in range(tmesh.n_elem):
        fs = tmesh.elem_faces[e]
        Ke = Ks[e]
        for a in range(tmesh.slots):
            for c in range(tmesh.slots):
                blk = Ke[a * b:(a + 1) * b, c * b:(c + 1) * b]
                key = (int(fs[a]), int(fs[c]))
                K[key] = K[key] + blk if key in K else blk.copy()
    R = np.array(G, dtype=np.float64, copy=True)
    for e in range(tmesh.n_elem):
        np.add.at(R, tmesh.element_dofs(e), rs[e])
    return K, R


def to_dense(tmesh, K):
    b = tmesh.b
    M = np.zeros((tmesh.n_trace, tmesh.n_trace))
    for (f, g), blk in K.items():
        M[f * b:(f + 1) * b, g * b:(g + 1) * b] = blk
    return M


def matvec(tmesh, K, x):
    b = tmesh.b
    y = np.zeros(tmesh.n_trace)
    for (f, g), blk in K.items():
        y[f * b:(f + 1) * b] += blk @ x[g * b:(g + 1) * b]
    return y
