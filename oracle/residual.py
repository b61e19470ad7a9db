"""Residual of the uncondensed Newton system (section 2.2.1).

Parity: pinned (tests compare with the residual of a dense assembled copy of
[A B; C D] on small meshes).

r_F,e = F_e - A_e z_e - B_e u_e per element;
r_G = G - sum_e P_e^T (C_e z_e + D_e u_e) over the trace.
Returns sqrt(sum ||r_F,e||^2 + ||r_G||^2) / sqrt(sum ||F_e||^2 + ||G||^2).
"""
import numpy as np


def full_residual(tmesh, blocks, G, z, uhat):
    rG = np.array(G, dtype=np.float64, copy=True)
    num = 0.0
    den = float(np.dot(G, G))
    for e, blk in enumerate(blocks):
        dofs = tmesh.element_dofs(e)
        ue = uhat[dofs]
        rF = blk["F"] - blk["A"] @ z[e] - blk["B"] @ ue
        num += float(rF @ rF)
        den += float(blk["F"] @ blk["F"])
        np.subtract.at(rG, dofs, blk["C"] @ z[e] + blk["D"] @ ue)
    num += float(rG @ rG)
    return np.sqrt(num / den), rG
