"""Element static condensation (section 2.2.1, eq. LS).

Parity: pinned.  Tests check it against a dense solve of the uncondensed
Newton system on small meshes, against the Schur determinant identity
det[A B; C D] = det(A) det(K_e), and against the first block row residual.

Per element e, with A_e factored by LAPACK getrf (partial pivoting):
  W = A_e^{-1} B_e,  w = A_e^{-1} F_e,
  K_e = D_e - C_e W,  r_e = -C_e w.
Summing P_e^T K_e P_e gives K = D - C A^{-1} B and G + sum P_e^T r_e gives
R = G - C A^{-1} F, since A is block diagonal.
"""
import numpy as np
import scipy.linalg as sla


def condense_element(A, B, C, D, F=None):
    lu = sla.lu_factor(A)
    W = sla.lu_solve(lu, B)
    Ke = D - C @ W
    if F is None:
        return Ke, None, lu
    w = sla.lu_solve(lu, F)
    re = -(C @ w)
    return Ke, re, lu


def condense_all(blocks):
    """blocks: iterable of dicts with A, B, C, D, F.  Returns (Ke list, re list)."""
    Ks, rs = [], []
    for blk in blocks:
        Ke, re, _ = condense_element(blk["A"], blk["B"], blk["C"], blk["D"], blk["F"])
        Ks.append(Ke)
        rs.append(re)
    return Ks, rs
