"""The Newton-step linear solve assembled from the C-ABI calls.

FP64 form (section 2.2): condense -> assemble -> BILU(0) -> GMRES -> recover
the element unknowns.

Mixed form: the same steps with FP32 (or BF16-operand) factors and FP32
blocks of K and of its BILU(0), followed by iterative refinement in FP64:
the residual of the uncondensed system is formed with the FP64 element
matrices, a correction is solved with the low-precision factors (right-hand
side condensation, GMRES on the FP32 trace system, back-substitution) and
added in FP64, until ||[F;G] - [A B; C D][z;u]|| / ||[F;G]|| <= tol.
"""
import math
import time

import torch

from . import api
from ._lib import F64, F32, BF16


class StepTimer:
    """Per-phase wall-clock via HIP events on the current stream."""

    def __init__(self, enabled=False):
        self.enabled = enabled
        self.events = []

    def mark(self, name):
        if self.enabled:
            ev = torch.cuda.Event(enable_timing=True)
            ev.record()
            self.events.append((name, ev))

    def phases(self):
        if not self.enabled or len(self.events) < 2:
            return {}
        torch.cuda.synchronize()
        out = {}
        for (n0, e0), (n1, e1) in zip(self.events[:-1], self.events[1:]):
            out[n1] = out.get(n1, 0.0) + e0.elapsed_time(e1)
        return out


class NewtonStepSolver:
    """Holds a mesh and the per-step device buffers of one simulation."""

    def __init__(self, ctx, mesh, n_local, restart=100, ordering="colour"):
        self.ctx = ctx
        self.mesh = mesh
        self.n = n_local
        self.restart = restart
        self.fac = None
        self.K = None
        self.M = None
        self.prec = None
        # the GMRES workspace, allocated once for every solve of this mesh
        self.gm = api.GmresState(ctx, mesh, restart)

    # -- factorisation (the part that depends on the matrices only) --------
    def factor(self, A, B, C, D, F=None, prec=F64, timer=None):
        ctx, mesh = self.ctx, self.mesh
        timer = timer or StepTimer(False)
        self.fac = api.condense(ctx, A, B, C, D, F, prec=prec, out=self.fac if self.prec == prec else None)
        timer.mark("condense")
        self.K, _ = api.assemble(ctx, mesh, Ke=self.fac["Ke"], prec=prec,
                                 Kbsr=self.K if self.prec == prec else None)
        timer.mark("assemble")
        self.M = api.factor_ilu0(ctx, mesh, self.K, prec=prec, Mbsr=self.M if self.prec == prec else None)
        timer.mark("factor_ilu0")
        self.prec = prec
        return self.fac

    def _trace_solve(self, R, rtol, max_iters=10000):
        return api.gmres_solve(self.ctx, self.mesh, self.K, self.M, R, self.restart, rtol, max_iters=max_iters,
                               kprec=self.prec, mprec=self.prec, state=self.gm)

    # -- FP64 form ----------------------------------------------------------
    def solve_fp64(self, A, B, C, D, F, G, rtol, timer=None):
        """Full FP64 Newton-step solve; returns (z, uhat, info)."""
        timer = timer or StepTimer(False)
        timer.mark("start")
        self.factor(A, B, C, D, F, prec=F64, timer=timer)
        _, R = api.assemble(self.ctx, self.mesh, r=self.fac["r"], G=G, prec=F64)
        timer.mark("assemble")
        uhat, info = self._trace_solve(R, rtol)
        timer.mark("gmres")
        z = api.backsolve_local(self.ctx, self.mesh, self.fac, uhat, prec=F64)
        timer.mark("backsolve")
        info["phases_ms"] = timer.phases()
        return z, uhat, info

    def solve_rhs_fp64(self, F, G, rtol):
        """New right-hand side with the retained FP64 factors."""
        w, r = api.condense_rhs(self.ctx, self.fac, F, prec=F64)
        _, R = api.assemble(self.ctx, self.mesh, r=r, G=G, prec=F64)
        uhat, info = self._trace_solve(R, rtol)
        z = api.backsolve_local(self.ctx, self.mesh, self.fac, uhat, prec=F64, w=w)
        return z, uhat, info

    # -- mixed form with FP64 refinement ----------------------------------
    def refine(self, A, B, C, D, F, G, z, uhat, tol, max_steps=30, timer=None, info=None):
        """FP64 iterative refinement of (z, uhat) with the low-precision factors."""
        ctx, mesh = self.ctx, self.mesh
        timer = timer or StepTimer(False)
        info = info if info is not None else {}
        hist = []
        steps = 0
        while True:
            rF, rG, sums = api.residual_full(ctx, mesh, A, B, C, D, F, G, z, uhat)
            s = sums.cpu()
            timer.mark("residual_fp64")
            rho = math.sqrt((s[0] + s[1]).item() / (s[2] + s[3]).item())
            hist.append(rho)
            if not math.isfinite(rho):
                raise api.IedgError(-4, "refinement residual is not finite")
            if rho <= tol or steps >= max_steps:
                break
            if len(hist) >= 3 and hist[-1] > 0.5 * hist[-2] and hist[-2] > 0.5 * hist[-3]:
                break  # stagnation
            w_c, r_c = api.condense_rhs(ctx, self.fac, rF, prec=self.prec)
            _, R_c = api.assemble(ctx, mesh, r=r_c, G=rG, prec=self.prec)
            crtol = max(1e-7, min(0.1, 0.1 * tol / rho))
            du, ginfo = self._trace_solve(R_c, crtol)
            dz = api.backsolve_local(ctx, mesh, self.fac, du, prec=self.prec, w=w_c)
            api.axpy(ctx, 1.0, du, uhat)
            api.axpy(ctx, 1.0, dz, z)
            info["iters"] = info.get("iters", 0) + ginfo["iters"]
            steps += 1
            timer.mark("correction")
        info["refine_steps"] = steps
        info["rho_hist"] = hist
        info["rho_full"] = hist[-1]
        info["converged_full"] = hist[-1] <= tol
        return z, uhat, info

    def solve_rhs_mixed(self, A, B, C, D, F, G, tol=1e-8, inner_rtol=1e-6):
        """New right-hand side with the retained low-precision factors, then
        FP64 refinement against the true element matrices."""
        w, r = api.condense_rhs(self.ctx, self.fac, F, prec=self.prec)
        _, R = api.assemble(self.ctx, self.mesh, r=r, G=G, prec=self.prec)
        uhat, info = self._trace_solve(R, inner_rtol)
        z = api.backsolve_local(self.ctx, self.mesh, self.fac, uhat, prec=self.prec, w=w)
        return self.refine(A, B, C, D, F, G, z, uhat, tol, info=info)

    def solve_mixed(self, A, B, C, D, F, G, tol=1e-8, prec=F32, inner_rtol=1e-6, timer=None):
        timer = timer or StepTimer(False)
        timer.mark("start")
        self.factor(A, B, C, D, F, prec=prec, timer=timer)
        _, R = api.assemble(self.ctx, self.mesh, r=self.fac["r"], G=G, prec=prec)
        timer.mark("assemble")
        uhat, info = self._trace_solve(R, inner_rtol)
        timer.mark("gmres")
        z = api.backsolve_local(self.ctx, self.mesh, self.fac, uhat, prec=prec)
        timer.mark("backsolve")
        z, uhat, info = self.refine(A, B, C, D, F, G, z, uhat, tol, timer=timer, info=info)
        info["phases_ms"] = timer.phases()
        return z, uhat, info
