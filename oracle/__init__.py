"""Plain FP64 CPU oracle for the IEDG Newton-step linear solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` use it.  It shares no code with the HIP path
(``paper_1605_01020_amd``); the only common dependency is the seeded input
generator package ``synth``, which holds none of the solver's arithmetic.

What it computes (Fernandez, Nguyen, Roca, Peraire, "Implicit large-eddy
simulation of compressible flows using the Interior Embedded Discontinuous
Galerkin method", section 2.2):

* the Newton system [A B; C D][dZ; dU] = [F; G] with block-diagonal A
  (section 2.2.1);
* static condensation K = D - C A^{-1} B, R = G - C A^{-1} F (eq. LS);
* left-preconditioned restarted GMRES with iterated classical Gram-Schmidt
  on M^{-1} K dU = M^{-1} R (section 2.2.2, eq. LS1);
* M = L~ U~, the zero-fill block incomplete LU (BILU(0)) of K under a given
  row ordering (section 2.2.2), and the minimum discarded fill ordering the
  paper applies to it;
* the restricted additive Schwarz preconditioner with delta-level overlap
  and BILU(0) subdomain solves (section 2.2.2), for N > 1 subdomains;
* recovery of the element unknowns dZ_e = A_e^{-1} (F_e - B_e dU_e), which
  the paper leaves implicit ("readily eliminated");
* the minimal-residual initial guess for Newton's method (section 2.2.1,
  eq. MinRes2): Levenberg-Marquardt with finite-difference gradients over
  combinations of previous solutions, on a synthetic nonlinear residual.

Every function is written for clarity, not speed.  Parity status of each
function is stated in its module docstring.
"""
from .mesh import TraceMesh
from .condense import condense_element, condense_all
from .assembly import assemble
from .ordering import natural_order, greedy_colour_order, level_sets
from .mdf import mdf_order
from .ras import ras_setup, ras_apply, overlap
from .bilu0 import bilu0, bilu0_apply
from .gmres import gmres
from .backsolve import backsolve_element, backsolve_all
from .residual import full_residual
from .solve import newton_step_solve
from .mr import mr_guess, nonlinear_residual

__all__ = [
    "TraceMesh", "condense_element", "condense_all", "assemble",
    "natural_order", "greedy_colour_order", "level_sets", "mdf_order", "ras_setup", "ras_apply", "overlap", "bilu0",
    "bilu0_apply", "gmres", "backsolve_element", "backsolve_all",
    "full_residual", "newton_step_solve",
]
