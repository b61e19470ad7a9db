"""Zero fill-in block incomplete LU, BILU(0) (section 2.2.2).

Parity: pinned.  Tests check the defining property of ILU(0), that the
product of the factors reproduces K on every block of K's pattern; that the
factors are the exact block LU when the pattern admits no fill
(block-tridiagonal matrices and the single-element mesh, whose six faces are
all coupled); and that point ILU(0) and block ILU(0) coincide.

Rows are eliminated in the given order.  For the row of face i and each
lower neighbour k (earlier in the order) taken in elimination order:
  L_ik = A_ik U_kk^{-1};
  A_ij -= L_ik U_kj  for every later j coupled to both i and k.
What is left on and right of the diagonal is U~.  The pivot blocks U_kk are
inverted exactly (dense LU with partial pivoting).
"""
import numpy as np
import scipy.linalg as sla


def bilu0(tmesh, K, order):
    """`order` lists the block rows to factor (all faces, or the faces of a
    subdomain whose pattern `tmesh` restricts to them)."""
    pos = np.full(tmesh.n_face, -1, dtype=np.int64)
    pos[np.asarray(order)] = np.arange(len(order))
    L, U = {}, {}
    Uinv = {}
    for i in order:
        i = int(i)
        row = {g: K[(i, g)].copy() for g in tmesh.pattern[i]}
        lower = sorted((g for g in row if pos[g] < pos[i]), key=lambda g: pos[g])
        for k in lower:
            Lik = row[k] @ Uinv[k]
            L[(i, k)] = Lik
            for j in row:
                if pos[j] > pos[k] and (k, j) in U:
                    row[j] -= Lik @ U[(k, j)]
        for g in row:
            if pos[g] >= pos[i]:
                U[(i, g)] = row[g]
        Uinv[i] = sla.lu_solve(sla.lu_factor(row[i]), np.eye(tmesh.b))
    return {"L": L, "U": U, "Uinv": Uinv, "order": np.asarray(order), "pos": pos}


def bilu0_apply(tmesh, fac, r):
    """z = (L~ U~)^{-1} r: unit block-lower sweep, then block-upper sweep."""
    b = tmesh.b
    order, pos = fac["order"], fac["pos"]
    y = np.array(r, dtype=np.float64, copy=True)
    for i in order:
        i = int(i)
        s = y[i * b:(i + 1) * b]
        for g in tmesh.pattern[i]:
            if pos[g] < pos[i]:
                s = s - fac["L"][(i, g)] @ y[g * b:(g + 1) * b]
        y[i * b:(i + 1) * b] = s
    x = y
    for i in order[::-1]:
        i = int(i)
        s = x[i * b:(i + 1) * b]
        for g in tmesh.pattern[i]:
            if pos[g] > pos[i]:
                s = s - fac["U"][(i, g)] @ x[g * b:(g + 1) * b]
        x[i * b:(i + 1) * b] = fac["Uinv"][i] @ s
    return x


def product_blocks(tmesh, fac):
    """(L~ U~)_{ij} for all face pairs (i, j) reachable through the factors."""
    pos = fac["pos"]
    out = {}
    for (i, j), Uij in fac["U"].items():
        out[(i, j)] = out.get((i, j), 0) + Uij
    for (i, k), Lik in fac["L"].items():
        for g in tmesh.pattern[k]:
            if (k, g) in fac["U"]:
                out[(i, g)] = out.get((i, g), 0) + Lik @ fac["U"][(k, g)]
    return out
