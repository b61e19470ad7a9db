"""Shared test helpers: seeded host inputs for a mesh case (synth only)."""
import numpy as np

from synth import StructuredHexMesh, ElementSpec, element_inputs, trace_rhs, SEED_BASE


def host_case(dims, p, seed=SEED_BASE, mesh_id=0, rhs=0):
    mesh = StructuredHexMesh(*dims)
    spec = ElementSpec(p)
    blocks = [element_inputs(spec, seed, mesh_id, e, rhs=rhs) for e in range(mesh.n_elem)]
    G = trace_rhs(spec, seed, mesh_id, mesh.n_face, rhs=rhs)
    return mesh, spec, blocks, G


def dense_uncondensed(tmesh, blocks, G):
    """The full Newton matrix [A B; C D] and right-hand side [F; G] as dense arrays."""
    n = blocks[0]["A"].shape[0]
    E, Nt = tmesh.n_elem, tmesh.n_trace
    M = np.zeros((E * n + Nt, E * n + Nt))
    rhs = np.zeros(E * n + Nt)
    for e, blk in enumerate(blocks):
        d = tmesh.element_dofs(e) + E * n
        loc = np.arange(e * n, (e + 1) * n)
        M[np.ix_(loc, loc)] = blk["A"]
        # add.at: in the IEDG numbering one element may map several local
        # trace dofs to the same global dof
        np.add.at(M, (loc[:, None], d[None, :]), blk["B"])
        np.add.at(M, (d[:, None], loc[None, :]), blk["C"])
        np.add.at(M, (d[:, None], d[None, :]), blk["D"])
        rhs[loc] = blk["F"]
    rhs[E * n:] = G
    return M, rhs
