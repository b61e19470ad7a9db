"""One Newton-step linear solve, end to end (sections 2.2.1 and 2.2.2).

Parity: pinned by the dense direct solve of the uncondensed system on small
meshes (tests).

Steps, in the paper's order: eliminate the element unknowns (K, R of eq. LS),
factor M = BILU(0)(K) under the given ordering, solve M^{-1} K u = M^{-1} R
by GMRES(m) with ICGS (eq. LS1), recover z_e.  On one subdomain the RAS
preconditioner is the BILU(0) of the whole K.
"""
import numpy as np

from .mesh import TraceMesh
from .condense import condense_all
from .assembly import assemble, matvec
from .ordering import greedy_colour_order, natural_order
from .bilu0 import bilu0, bilu0_apply
from .gmres import gmres
from .backsolve import backsolve_all
from .residual import full_residual


def newton_step_solve(tmesh, blocks, G, restart, rtol, order="colour",
                      inner_factor=0.1, max_cycles=200, precond=True):
    Ks, rs = condense_all(blocks)
    K, R = assemble(tmesh, Ks, rs, G)
    if isinstance(order, str):
        order = greedy_colour_order(tmesh) if order == "colour" else natural_order(tmesh)
    Kmv = lambda v: matvec(tmesh, K, v)
    if precond:
        fac = bilu0(tmesh, K, order)
        Minv = lambda v: bilu0_apply(tmesh, fac, v)
    else:
        fac = None
        Minv = lambda v: np.array(v, copy=True)
    uhat, info = gmres(Kmv, Minv, R, restart, rtol, max_cycles=max_cycles,
                       inner_factor=inner_factor)
    z = backsolve_all(tmesh, blocks, uhat)
    rho_full, _ = full_residual(tmesh, blocks, G, z, uhat)
    info["rho_full"] = rho_full
    return {"uhat": uhat, "z": z, "K": K, "R": R, "Ks": Ks, "rs": rs,
            "fac": fac, "order": order, "info": info}
