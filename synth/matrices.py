"""Seeded element blocks of the Newton system and the workload table.

Block roles follow the Newton linear system of the paper (section 2.2.1):
per element e, A_e couples the element's (q, u) dofs, B_e couples them to the
trace dofs of its six faces, C_e and D_e are the trace-equation blocks, F_e
and G are the right-hand sides.  The synthetic distributions are

  A_e = 2 I + N(0, 1/n),   B_e, C_e ~ N(0, 0.1/n),
  D_e = 1.5 I + N(0, 0.05/b)  (all 36 face-pair blocks),   F_e, G ~ N(0, 1),

with N(0, v) meaning variance v, n = 20 (p+1)^3 local dofs, b = 5 (p+1)^2 dofs
per face and t = 6 b trace dofs per element.  Matrices are row-major.

Stream ids: entry e (row-major) of matrix X of element el uses Philox
counter (lo(e>>1), hi(e>>1), el, tag), tag = mesh_id << 20 | X << 16 | rhs,
X = 1..6 for A, B, C, D, F, G; G uses element id 0xFFFFFFFF and the global
trace dof index.  The key is the 64-bit seed SEED_BASE + config index.
"""
from dataclasses import dataclass, field
import math
import numpy as np

from .philox import normals, philox4x32_10
from .mesh import StructuredHexMesh

SEED_BASE = 1605010200
MAT_A, MAT_B, MAT_C, MAT_D, MAT_F, MAT_G = 1, 2, 3, 4, 5, 6
G_STREAM = 0xFFFFFFFF
DRAW_STREAM = 0xFFFFFFFE


def make_tag(mesh_id, mat, rhs=0):
    return ((mesh_id & 0xFFF) << 20) | ((mat & 0xF) << 16) | (rhs & 0xFFFF)


@dataclass(frozen=True)
class ElementSpec:
    """Sizes for polynomial degree p with 5 conserved variables in 3-D."""
    p: int

    @property
    def n(self):  # (u, q): 5 + 15 components at (p+1)^3 nodes
        return 20 * (self.p + 1) ** 3

    @property
    def b(self):  # 5 components at (p+1)^2 face nodes
        return 5 * (self.p + 1) ** 2

    @property
    def t(self):
        return 6 * self.b


# (name, diagonal, variance as a function of the spec)
_DISTS = {
    MAT_A: (2.0, lambda s: 1.0 / s.n),
    MAT_B: (0.0, lambda s: 0.1 / s.n),
    MAT_C: (0.0, lambda s: 0.1 / s.n),
    MAT_D: (1.5, lambda s: 0.05 / s.b),
    MAT_F: (0.0, lambda s: 1.0),
    MAT_G: (0.0, lambda s: 1.0),
}


def dist_params(spec, mat):
    diag, var = _DISTS[mat]
    return diag, math.sqrt(var(spec))


def _matrix(spec, seed, mesh_id, elem, mat, rows, cols, rhs=0):
    diag, sigma = dist_params(spec, mat)
    z = normals(0, rows * cols, elem, make_tag(mesh_id, mat, rhs), seed)
    m = (sigma * z).reshape(rows, cols)
    if diag != 0.0:
        m[np.arange(rows), np.arange(rows)] += diag
    return m


def element_inputs(spec, seed, mesh_id, elem, rhs=0, which="ABCDF"):
    """Host copies of the element blocks; returns a dict keyed by letter."""
    n, t = spec.n, spec.t
    out = {}
    if "A" in which:
        out["A"] = _matrix(spec, seed, mesh_id, elem, MAT_A, n, n)
    if "B" in which:
        out["B"] = _matrix(spec, seed, mesh_id, elem, MAT_B, n, t)
    if "C" in which:
        out["C"] = _matrix(spec, seed, mesh_id, elem, MAT_C, t, n)
    if "D" in which:
        out["D"] = _matrix(spec, seed, mesh_id, elem, MAT_D, t, t)
    if "F" in which:
        out["F"] = _matrix(spec, seed, mesh_id, elem, MAT_F, n, 1, rhs).ravel()
    return out


def trace_rhs(spec, seed, mesh_id, n_face, rhs=0, first=0, count=None):
    """Global trace right-hand side G (length n_face * b), or a slice of it."""
    total = n_face * spec.b
    count = total - first if count is None else count
    return normals(first, count, G_STREAM, make_tag(mesh_id, MAT_G, rhs), seed)


@dataclass
class MeshCase:
    mesh_id: int
    dims: tuple
    p: int

    @property
    def spec(self):
        return ElementSpec(self.p)

    @property
    def mesh(self):
        return StructuredHexMesh(*self.dims)


@dataclass
class Workload:
    """One benchmark/test configuration: meshes, seed, solver settings."""
    name: str
    seed: int
    meshes: list
    restart: int
    rtol: float
    n_rhs: int = 1
    extra: dict = field(default_factory=dict)


BATCH_SHAPES = [(4, 4, 4), (6, 6, 6), (8, 8, 4), (12, 12, 6)]


def draw_meshes(seed, count):
    """Mesh shape and degree per index: shape = x0 mod 4, p = 2 + x1 mod 3."""
    idx = np.arange(count, dtype=np.uint64)
    x0, x1, _, _ = philox4x32_10(idx, 0, DRAW_STREAM, 0, seed & 0xFFFFFFFF,
                                 seed >> 32)
    return [MeshCase(i, BATCH_SHAPES[int(x0[i]) % 4], 2 + int(x1[i]) % 3)
            for i in range(count)]


def workload(config):
    """The five standard configurations, by index."""
    seed = SEED_BASE + config
    if config == 0:
        return Workload("cfg0_fp64_4x4x4_p2", seed, [MeshCase(0, (4, 4, 4), 2)],
                        restart=50, rtol=1e-10)
    if config == 1:
        return Workload("cfg1_fp64_16x16x8_p3", seed, [MeshCase(0, (16, 16, 8), 3)],
                        restart=100, rtol=1e-10, n_rhs=10)
    if config == 2:
        return Workload("cfg2_mixed_16x16x8_p3", seed, [MeshCase(0, (16, 16, 8), 3)],
                        restart=100, rtol=1e-8, n_rhs=10)
    if config == 3:
        return Workload("cfg3_batch24", seed, draw_meshes(seed, 24),
                        restart=100, rtol=1e-8)
    if config == 4:
        return Workload("cfg4_serving64", seed, draw_meshes(seed, 64),
                        restart=100, rtol=1e-8)
    raise ValueError(config)
