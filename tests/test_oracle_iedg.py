"""Pins of the IEDG trace numbering (synth.StructuredHexMesh.iedg_trace_nodes,
section 2.1: the trace space is continuous on interior faces and
discontinuous on boundary faces) and of the oracle's Newton-step solve on
it: closed-form node counts, sharing multiplicities, continuity where an
element's own faces meet, the condensed solve against the dense uncondensed
system, and the smaller trace system the paper attributes to IEDG."""
import numpy as np
import pytest

import oracle
from oracle.assembly import matvec
from synth import StructuredHexMesh, ElementSpec, element_inputs, trace_rhs, SEED_BASE

from helpers import dense_uncondensed


def _closed_form_nodes(nx, ny, nz, p):
    """Interior-face lattice points by inclusion-exclusion over the interior
    planes, plus (p+1)^2 private nodes per boundary face."""
    X, Y, Z = p * nx + 1, p * ny + 1, p * nz + 1
    ix, iy, iz = nx - 1, ny - 1, nz - 1
    planes = ix * Y * Z + iy * X * Z + iz * X * Y
    lines = ix * iy * Z + ix * iz * Y + iy * iz * X
    points = ix * iy * iz
    bfaces = 2 * (ny * nz + nx * nz + nx * ny)
    return planes - lines + points + bfaces * (p + 1) ** 2


@pytest.mark.parametrize("dims,p", [((1, 1, 1), 1), ((2, 1, 1), 2), ((2, 2, 2), 1), ((3, 2, 2), 3), ((2, 3, 4), 2)])
def test_node_count_closed_form(dims, p):
    m = StructuredHexMesh(*dims)
    en, n_nodes = m.iedg_trace_nodes(p)
    assert en.shape == (m.n_elem, 6 * (p + 1) ** 2)
    assert n_nodes == _closed_form_nodes(*dims, p)
    assert sorted(set(en.ravel().tolist())) == list(range(n_nodes))


def test_sharing_and_continuity():
    p = 2
    m = StructuredHexMesh(3, 3, 3)
    en, n_nodes = m.iedg_trace_nodes(p)
    p1 = p + 1
    elems_of = [set() for _ in range(n_nodes)]
    for e in range(m.n_elem):
        for v in en[e]:
            elems_of[v].add(e)
    # the centre element (1,1,1): its corner nodes are interior lattice
    # vertices shared by 8 elements, edge-interior nodes by 4, face-interior by 2
    e = (1 * 3 + 1) * 3 + 1
    faces = en[e].reshape(6, p1, p1)
    assert len(elems_of[faces[0, 0, 0]]) == 8
    assert len(elems_of[faces[0, 1, 0]]) == 4
    assert len(elems_of[faces[0, 1, 1]]) == 2
    # continuity where the element's own faces meet: -x face (u=y, v=z) and
    # -y face (u=x, v=z) share the edge x = x0, y = y0 along z
    assert np.array_equal(faces[0][0, :], faces[2][0, :])
    # -x face and -z face (u=x, v=y) share the edge x = x0, z = z0 along y
    assert np.array_equal(faces[0][:, 0], faces[4][0, :])
    assert len(set(en[e].tolist())) == (p + 1) ** 3 - (p - 1) ** 3
    # a corner element: its three boundary faces have private nodes
    ef = m.elem_faces()
    d, idx = m.face_geometry()
    for a in (0, 2, 4):
        f = ef[0, a]
        assert idx[f] == 0
        for v in en[0].reshape(6, p1 * p1)[a]:
            assert elems_of[v] == {0}


def _iedg_case(dims, p, seed=SEED_BASE + 21):
    hm = StructuredHexMesh(*dims)
    spec = ElementSpec(p)
    en, n_nodes = hm.iedg_trace_nodes(p)
    tm = oracle.TraceMesh(en, n_nodes, 5)
    blocks = [element_inputs(spec, seed, 0, e) for e in range(hm.n_elem)]
    G = trace_rhs(spec, seed, 0, hm.n_face, count=n_nodes * 5)
    return hm, spec, tm, blocks, G


@pytest.mark.parametrize("dims,p", [((2, 1, 1), 1), ((2, 2, 1), 2)])
def test_condensed_solve_equals_dense_uncondensed(dims, p):
    hm, spec, tm, blocks, G = _iedg_case(dims, p)
    assert tm.t == spec.t
    M, rhs = dense_uncondensed(tm, blocks, G)
    x = np.linalg.solve(M, rhs)
    Ks, rs = oracle.condense_all(blocks)
    K, R = oracle.assemble(tm, Ks, rs, G)
    from oracle.assembly import to_dense
    u = np.linalg.solve(to_dense(tm, K), R)
    z = np.stack(oracle.backsolve_all(tm, blocks, u))
    E, n = tm.n_elem, spec.n
    assert np.linalg.norm(u - x[E * n:]) <= 1e-10 * np.linalg.norm(x[E * n:])
    assert np.linalg.norm(z.ravel() - x[:E * n]) <= 1e-10 * np.linalg.norm(x[:E * n])
    rho, _ = oracle.full_residual(tm, blocks, G, z, u)
    assert rho <= 1e-12


def test_iedg_system_smaller_than_face_private():
    """The trace system of the IEDG numbering has fewer unknowns and fewer
    nonzeros than the face-private one (the paper's point about K)."""
    p = 3
    hm = StructuredHexMesh(4, 4, 4)
    en, n_nodes = hm.iedg_trace_nodes(p)
    tn = oracle.TraceMesh(en, n_nodes, 5)
    tf = oracle.TraceMesh(hm.elem_faces(), hm.n_face, 5 * (p + 1) ** 2)
    # 4x4x4 elements, p = 3: 0.71 of the unknowns, 0.55 of the nonzeros (the
    # ratios fall further as the share of boundary faces drops)
    assert tn.n_trace < 0.75 * tf.n_trace
    assert tn.nnzb() * 25 < 0.6 * tf.nnzb() * tf.b ** 2


def test_iedg_newton_step_solve_converges():
    hm, spec, tm, blocks, G = _iedg_case((2, 2, 1), 1)
    res = oracle.newton_step_solve(tm, blocks, G, restart=100, rtol=1e-12)
    M, rhs = dense_uncondensed(tm, blocks, G)
    x = np.linalg.solve(M, rhs)
    E, n = tm.n_elem, spec.n
    assert np.linalg.norm(res["uhat"] - x[E * n:]) <= 1e-9 * np.linalg.norm(x[E * n:])
