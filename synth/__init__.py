"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package holds input generation only: the structured hex mesh topology
(element -> face incidence) and counter-based random element matrices.  It
contains none of the solver's arithmetic.  The host generator (numpy) feeds
the oracle; the device generator (``libsynth.so``, built from
``synth/csrc/synth_gen.hip``) writes the same values straight into HBM for
the GPU path.  Both implement Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11) with a Box-Muller
transform.
"""
from .philox import philox4x32_10, uniforms53, normals
from .mesh import StructuredHexMesh
from .matrices import ElementSpec, Workload, element_inputs, trace_rhs, SEED_BASE

__all__ = [
    "philox4x32_10", "uniforms53", "normals", "StructuredHexMesh",
    "ElementSpec", "Workload", "element_inputs", "trace_rhs", "SEED_BASE",
]
