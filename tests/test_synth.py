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


def test_elementary_functions_of_the_generator():
    """ln_unit and cos_sin_turns (the generator's own series) against
    numpy's library functions to a few ulps, exact special values, and
    constants that are the nearest doubles to their exact values."""
    import math
    import re
    from decimal import Decimal, getcontext
    from fractions import Fraction
    from synth import philox as P
    getcontext().prec = 50
    ln2 = Decimal(2).ln()
    assert abs(Decimal(P.LN2) - ln2) <= Decimal(2.0 ** -53) * Decimal(P.LN2) / 2
    assert P.HALF_PI == math.pi / 2 and P.SQRT_HALF == math.sqrt(0.5)
    for k, c in enumerate(P.LOG_COEF):
        assert Fraction(c) == Fraction(float(Fraction(1, 2 * k + 1)))
        assert abs(Fraction(c) - Fraction(1, 2 * k + 1)) <= Fraction(c) * Fraction(1, 2 ** 53)
    for k, c in enumerate(P.SIN_COEF):
        exact = Fraction((-1) ** k, math.factorial(2 * k + 1))
        assert abs(Fraction(c) - exact) <= abs(exact) * Fraction(1, 2 ** 53)
    for k, c in enumerate(P.COS_COEF):
        exact = Fraction((-1) ** k, math.factorial(2 * k))
        assert abs(Fraction(c) - exact) <= abs(exact) * Fraction(1, 2 ** 53)
    rng = np.random.default_rng(4)
    u1 = (rng.integers(0, 2 ** 53, 200_000).astype(np.float64) + 1.0) * 2.0 ** -53
    ref = np.log(u1)
    assert np.all(np.abs(P.ln_unit(u1) - ref) <= 4.5e-16 * np.abs(ref) + 1e-300)
    u2 = rng.integers(0, 2 ** 53, 200_000).astype(np.float64) * 2.0 ** -53
    c, s = P.cos_sin_turns(u2)
    assert np.max(np.abs(c - np.cos(2 * np.pi * u2))) <= 1e-15
    assert np.max(np.abs(s - np.sin(2 * np.pi * u2))) <= 1e-15
    assert np.max(np.abs(c * c + s * s - 1.0)) <= 4.5e-16
    # exact values: ln 1 = 0, ln 2^-k = -k ln 2 (one rounding), quarter turns
    assert P.ln_unit(np.array([1.0]))[0] == 0.0
    for k in (1, 2, 17, 53):
        assert P.ln_unit(np.array([2.0 ** -k]))[0] == -k * P.LN2
    c, s = P.cos_sin_turns(np.array([0.0, 0.25, 0.5, 0.75]))
    assert np.array_equal(c, [1.0, 0.0, -1.0, 0.0]) and np.array_equal(s, [0.0, 1.0, 0.0, -1.0])
    # the device generator holds the same constants
    src = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                            "synth", "csrc", "synth_gen.hip")).read()
    def table(name):
        body = re.search(name + r"\[\d+\] = \{([^}]*)\}", src).group(1)
        return tuple(float.fromhex(x) for x in re.findall(r"-?0x[0-9a-f.]+p[-+]\d+", body))
    assert table("LOG_COEF") == P.LOG_COEF
    assert table("SIN_COEF") == P.SIN_COEF
    assert table("COS_COEF") == P.COS_COEF
    for name in ("LN2", "HALF_PI", "SQRT_HALF"):
        lit = re.search(r"constexpr double " + name + r" = (-?0x[0-9a-f.]+p[-+]\d+);", src).group(1)
        assert float.fromhex(lit) == getattr(P, name)


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
