"""Pins for the seeded input generator (host side) and the mesh numbering."""
import os

import numpy as np
import pytest

from synth import StructuredHexMesh, ElementSpec, element_inputs, trace_rhs, SEED_BASE
from synth.philox import philox4x32_10, uniforms53, normals
from synth.matrices import draw_meshes, workload, BATCH_SHAPES

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = philox4x32_10(v[0], v[1], v[2], v[3], v[4], v[5])
        assert [int(o) for o in out] == v[6:10]


def test_uniform_endpoints():
    z = np.uint32(0)
    o = np.uint32(0xFFFFFFFF)
    u1, u2 = uniforms53(z, z, z, z)
    assert u1 == 2.0 ** -53 and u2 == 0.0
    u1, u2 = uniforms53(o, o, o, o)
    assert u1 == 1.0 and u2 == 1.0 - 2.0 ** -53


def test_normal_moments():
    n = 400_000
    z = normals(0, n, 3, 11, SEED_BASE)
    se = 1.0 / np.sqrt(n)
    assert abs(z.mean()) < 5 * se
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0) * se
    assert abs(np.mean(z ** 4) - 3.0) < 5 * np.sqrt(96.0) * se
    # slices of a stream are the same numbers as the whole stream
    assert np.array_equal(normals(1001, 77, 3, 11, SEED_BASE), z[1001:1078])


def test_element_block_distributions():
    spec = ElementSpec(1)
    blk = element_inputs(spec, SEED_BASE, 0, 5)
    n, t, b = spec.n, spec.t, spec.b
    A = blk["A"]
    off = A[~np.eye(n, dtype=bool)]
    assert abs(np.diag(A).mean() - 2.0) < 5 * np.sqrt(1.0 / n / n)
    assert abs(off.var() * n - 1.0) < 0.05
    assert abs(blk["B"].var() * n / 0.1 - 1.0) < 0.05
    assert abs(blk["C"].var() * n / 0.1 - 1.0) < 0.05
    D = blk["D"]
    assert abs(np.diag(D).mean() - 1.5) < 0.05
    assert abs(D[~np.eye(t, dtype=bool)].var() * b / 0.05 - 1.0) < 0.1
    # distinct elements, matrices and right-hand sides draw distinct streams
    other = element_inputs(spec, SEED_BASE, 0, 6)
    assert not np.allclose(other["A"], A)
    f1 = element_inputs(spec, SEED_BASE, 0, 5, rhs=1, which="F")["F"]
    assert not np.allclose(f1, blk["F"])


def test_mesh_counts_closed_form():
    for dims in [(1, 1, 1), (2, 3, 4), (4, 4, 4), (16, 16, 8)]:
        m = StructuredHexMesh(*dims)
        nx, ny, nz = dims
        assert m.n_face == (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1)
        ef = m.elem_faces()
        counts = np.bincount(ef.ravel(), minlength=m.n_face)
        boundary = 2 * (ny * nz + nx * nz + nx * ny)
        assert (counts == 1).sum() == boundary
        assert (counts == 2).sum() == m.n_face - boundary
        assert counts.max() <= 2
        # every element has six distinct faces; opposite faces share the direction
        d, idx = m.face_geometry()
        assert (np.sort(ef, axis=1)[:, 1:] != np.sort(ef, axis=1)[:, :-1]).all()
        assert (d[ef] == np.array([0, 0, 1, 1, 2, 2])).all()
        assert (idx[ef[:, 1::2]] == idx[ef[:, 0::2]] + 1).all()


def test_config_draws_deterministic():
    a = draw_meshes(SEED_BASE + 3, 24)
    b = draw_meshes(SEED_BASE + 3, 24)
    assert [(m.dims, m.p) for m in a] == [(m.dims, m.p) for m in b]
    assert {m.dims for m in a} <= set(BATCH_SHAPES)
    assert {m.p for m in a} <= {2, 3, 4}
    assert len({m.p for m in a}) == 3
    w1 = workload(1)
    assert w1.meshes[0].dims == (16, 16, 8) and w1.meshes[0].p == 3
    assert w1.meshes[0].spec.n == 1280 and w1.meshes[0].spec.b == 80
