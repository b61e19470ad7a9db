"""Recovery of the element unknowns (section 2.2.1).

Parity: pinned by the first block row of the Newton system: tests check
F_e - A_e dZ_e - B_e dU_e = 0 to rounding.

The paper eliminates dZ element by element and leaves its recovery implicit;
from the first block row A dZ + B dU = F and block-diagonal A:
  dZ_e = A_e^{-1} (F_e - B_e dU_e).
"""
import scipy.linalg as sla


def backsolve_element(A, B, F, uhat_e, lu=None):
    lu = sla.lu_factor(A) if lu is None else lu
    return sla.lu_solve(lu, F - B @ uhat_e)


def backsolve_all(tmesh, blocks, uhat):
    return [backsolve_element(blk["A"], blk["B"], blk["F"], uhat[tmesh.element_dofs(e)])
            for e, blk in enumerate(blocks)]
