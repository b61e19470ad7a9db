"""MI355X (gfx950) implementation of the linear solve of one IEDG Newton step.

Fernandez, Nguyen, Roca, Peraire, section 2.2: element static condensation,
assembly of the trace system, BILU(0), left-preconditioned GMRES(m) with
iterated classical Gram-Schmidt, and element back-substitution.  The kernels
live in libiedg.so (C ABI: include/iedg.h); this package only marshals
arguments.
"""
from ._lib import F64, F32, BF16, LIB_PATH

__all__ = ["F64", "F32", "BF16", "LIB_PATH"]
