"""Batched form of the Newton-step linear solve: several meshes of uneven
size and polynomial degree solved together (section 2.2 for every mesh).

Per memory group of meshes:
  * condensation (section 2.2.1, eq. LS) of every element of every mesh in
    the group by ONE launch per element size (n, t): the work list
    interleaves (mesh, element) items, so small and large meshes share the
    chip, and the hardware dispatcher hands the next item to whichever CU
    finishes first;
  * per mesh: assembly, BILU(0) of the low-precision trace matrix, one
    device-driven GMRES cycle (section 2.2.2, eq. LS1), local
    back-substitution, then a fixed number of FP64 refinement steps
    (residual of the uncondensed system with the FP64 element matrices,
    correction with the retained low-precision factors);
  * the whole sequence is enqueued without host synchronisation, captured
    once in a HIP graph (torch.cuda.CUDAGraph drives hipGraph) and replayed.
After the replay the host reads each mesh's FP64 residual; a mesh that has
not reached the tolerance continues with eager refinement steps.

Inputs that do not fit at once are processed in groups whose resident bytes
stay under a budget; the element matrices of a group are generated on the
device before its graph runs.
"""
import math
import time
from dataclasses import dataclass, field

import torch

from . import api
from ._lib import F64, F32


def _esize(prec):
    return 8 if prec == F64 else 4


def sim_bytes(E, n, t, n_face, b, nnzb, prec, restart, n_stages):
    """Device bytes held by one simulation (inputs, factors, trace system,
    Krylov states and vectors)."""
    es = _esize(prec)
    N_t = n_face * b
    inputs = 8 * E * (n * n + 2 * n * t + t * t + n)
    factors = es * E * (n * n + 2 * n * t + t * t) + 4 * E * n + 8 * E * (n + t)
    trace = 2 * es * nnzb * b * b + 8 * N_t * 8
    krylov = n_stages * 8 * (restart + 3) * ((N_t + 63) // 64 * 64)
    local = 8 * E * n * 4 + 8 * E * t * 2
    return inputs + factors + trace + krylov + local


@dataclass
class SimResult:
    mesh_id: int
    iters: list = field(default_factory=list)
    rho_hist: list = field(default_factory=list)
    eager_steps: int = 0
    converged: bool = False


class Simulation:
    """Device state of one simulation: its trace mesh, FP64 element matrices
    and right-hand sides, low-precision factors and trace system, and the
    buffers of the solve and of its refinement."""

    def __init__(self, ctx, case, seed, prec=F32, restart=100, n_refine=1, tol=1e-8, inner_rtol=1e-6,
                 correction_rtol=1e-3, ordering="colour", cycle_steps=24, allocate=True):
        """The mesh and the GMRES workspaces are created here and kept for the
        simulation's lifetime; the per-solve arrays (inputs, factors, trace
        system, vectors) live in one byte arena that attach() carves up and
        detach() hands back (allocate=False: no arena yet)."""
        from synth.mesh import StructuredHexMesh
        self.ctx, self.case, self.seed, self.prec = ctx, case, seed, prec
        self.tol, self.inner_rtol, self.correction_rtol = tol, inner_rtol, correction_rtol
        self.n_refine = n_refine
        spec = case.spec
        hm = StructuredHexMesh(*case.dims)
        self.spec = spec
        self.E, self.n, self.t, self.b = hm.n_elem, spec.n, spec.t, spec.b
        self.mesh = api.Mesh(ctx, hm.elem_faces(), hm.n_face, spec.b, ordering=ordering)
        # device-driven cycles stop at cycle_steps Arnoldi steps (every step
        # is enqueued, later ones return at once after convergence); a cycle
        # that stops unconverged is continued by the refinement on the host
        # (corrections at tolerance 1e-3 need a few steps: half the cap)
        self.gm = [api.GmresState(ctx, self.mesh, min(restart, cycle_steps if s == 0 else max(8, cycle_steps // 2)))
                   for s in range(n_refine + 1)]
        self.restart = restart
        self.arena = None
        if allocate:
            self.attach(torch.empty(self.arena_bytes(), dtype=torch.uint8, device="cuda"))

    def _layout(self):
        """(name, shape, dtype) of every per-solve array."""
        E, n, t, N_t = self.E, self.n, self.t, self.mesh.n_trace
        f64, i32, lo = torch.float64, torch.int32, api.PREC_DTYPE[self.prec]
        return [("A", (E, n, n), f64), ("B", (E, n, t), f64), ("C", (E, t, n), f64), ("D", (E, t, t), f64),
                ("F", (E, n), f64), ("G", (N_t,), f64),
                ("LU", (E, n, n), lo), ("perm", (E, n), i32), ("U12", (E, n, t), lo), ("L21", (E, t, n), lo),
                ("Ke", (E, t, t), lo), ("w", (E, n), f64), ("r", (E, t), f64),
                ("K", (self.mesh.nnzb, self.b, self.b), lo), ("M", (self.mesh.nnzb, self.b, self.b), lo),
                ("R", (N_t,), f64), ("uhat", (N_t,), f64), ("z", (E, n), f64), ("rF", (E, n), f64),
                ("rG", (N_t,), f64), ("wc", (E, n), f64), ("rc", (E, t), f64), ("Rc", (N_t,), f64),
                ("du", (N_t,), f64), ("dz", (E, n), f64), ("sums", (self.n_refine + 1, 4), f64)]

    @staticmethod
    def _nbytes(shape, dtype):
        k = 1
        for d in shape:
            k *= d
        return k * torch.empty((), dtype=dtype).element_size()

    def arena_bytes(self):
        return sum((self._nbytes(sh, dt) + 255) // 256 * 256 for _, sh, dt in self._layout())

    def attach(self, arena):
        """Carve the per-solve arrays out of `arena` (a uint8 device tensor of
        at least arena_bytes(), every array on a 256-byte boundary)."""
        if arena.numel() < self.arena_bytes():
            raise ValueError("arena too small")
        views, off = {}, 0
        for name, shape, dt in self._layout():
            nb = self._nbytes(shape, dt)
            views[name] = arena[off:off + nb].view(dt).view(shape)
            off += (nb + 255) // 256 * 256
        self.arena = arena
        self.inp = {k: views[k] for k in "ABCDF"}
        self.G = views["G"]
        self.fac = {k: views[k] for k in ("LU", "perm", "U12", "L21", "Ke", "w", "r")}
        for k in ("K", "M", "R", "uhat", "z", "rF", "rG", "wc", "rc", "Rc", "du", "dz", "sums"):
            setattr(self, k, views[k])
        self.sums.zero_()

    def detach(self):
        """Give the arena back (the simulation keeps its mesh and workspaces)."""
        arena = self.arena
        self.arena = None
        for k in ("inp", "G", "fac", "K", "M", "R", "uhat", "z", "rF", "rG", "wc", "rc", "Rc", "du", "dz", "sums"):
            if hasattr(self, k):
                delattr(self, k)
        return arena

    def static_bytes(self):
        """Device bytes held for the whole lifetime (the GMRES workspaces; the
        mesh's index arrays and residual scratch are small beside them)."""
        ldv = (self.mesh.n_trace + 63) // 64 * 64
        return sum(8 * (g.steps + 3) * ldv for g in self.gm)

    @staticmethod
    def footprint(case, prec=F32, restart=100, n_refine=1):
        from synth.mesh import StructuredHexMesh
        hm = StructuredHexMesh(*case.dims)
        s = case.spec
        nnzb = _nnzb_estimate(hm)
        return sim_bytes(hm.n_elem, s.n, s.t, hm.n_face, s.b, nnzb, prec, restart, n_refine + 1)

    def generate(self, rhs=0):
        """Element matrices and right-hand sides on the device (seeded)."""
        from synth import device as sdev
        sdev.gen_blocks(self.spec, self.seed, self.case.mesh_id, self.E, which="ABCD", out=self.inp)
        self.set_rhs(rhs)

    def set_rhs(self, rhs):
        from synth import device as sdev
        sdev.gen_blocks(self.spec, self.seed, self.case.mesh_id, self.E, which="F", rhs=rhs, out=self.inp)
        sdev.gen_trace_rhs(self.spec, self.seed, self.case.mesh_id, self.mesh.n_face, rhs=rhs, out=self.G)

    def condense_segment(self):
        return (self.inp, self.fac)

    # -- enqueue (no host synchronisation) ---------------------------------
    def enqueue_after_condense(self):
        """Trace system, BILU(0), GMRES, back-substitution and refinement."""
        ctx, mesh, p = self.ctx, self.mesh, self.prec
        api.assemble(ctx, mesh, Ke=self.fac["Ke"], r=self.fac["r"], G=self.G, prec=p, Kbsr=self.K, R=self.R)
        api.factor_ilu0(ctx, mesh, self.K, prec=p, Mbsr=self.M)
        self._enqueue_solve(self.fac["w"], self.R, self.inner_rtol)

    def enqueue_factor(self):
        """Condensation of the matrices alone (no right-hand side), assembly
        of K and its BILU(0): the state a later enqueue_rhs() reuses."""
        ctx, mesh, p, i = self.ctx, self.mesh, self.prec, self.inp
        api.condense(ctx, i["A"], i["B"], i["C"], i["D"], None, prec=p, out=self.fac)
        api.assemble(ctx, mesh, Ke=self.fac["Ke"], prec=p, Kbsr=self.K)
        api.factor_ilu0(ctx, mesh, self.K, prec=p, Mbsr=self.M)

    def enqueue_rhs(self):
        """New right-hand side with the retained factors (factors resident)."""
        ctx, mesh, p = self.ctx, self.mesh, self.prec
        api.condense_rhs(ctx, self.fac, self.inp["F"], prec=p, w=self.fac["w"], r=self.fac["r"])
        api.assemble(ctx, mesh, r=self.fac["r"], G=self.G, prec=p, R=self.R)
        self._enqueue_solve(self.fac["w"], self.R, self.inner_rtol)

    def _enqueue_solve(self, w, R, rtol):
        ctx, mesh, p = self.ctx, self.mesh, self.prec
        self.gm[0].enqueue(self.K, self.M, R, self.uhat, rtol, kprec=p, mprec=p)
        api.backsolve_local(ctx, mesh, self.fac, self.uhat, prec=p, w=w, z=self.z)
        for s in range(self.n_refine):
            self._enqueue_residual(s)
            self._enqueue_correction(self.gm[s + 1])
        self._enqueue_residual(self.n_refine)

    def _enqueue_residual(self, slot):
        i = self.inp
        api.residual_full(self.ctx, self.mesh, i["A"], i["B"], i["C"], i["D"], i["F"], self.G, self.z, self.uhat,
                          rF=self.rF, rG=self.rG, sums=self.sums[slot])

    def _enqueue_correction(self, gm, rtol=None):
        ctx, mesh, p = self.ctx, self.mesh, self.prec
        api.condense_rhs(ctx, self.fac, self.rF, prec=p, w=self.wc, r=self.rc)
        api.assemble(ctx, mesh, r=self.rc, G=self.rG, prec=p, R=self.Rc)
        gm.enqueue(self.K, self.M, self.Rc, self.du, self.correction_rtol if rtol is None else rtol,
                   kprec=p, mprec=p)
        api.backsolve_local(ctx, mesh, self.fac, self.du, prec=p, w=self.wc, z=self.dz)
        api.axpy(ctx, 1.0, self.du, self.uhat)
        api.axpy(ctx, 1.0, self.dz, self.z)

    # -- host side ----------------------------------------------------------
    @staticmethod
    def _rho(s):
        den = s[2] + s[3]
        return math.sqrt((s[0] + s[1]) / den) if den > 0 else 0.0

    def finish(self, max_eager=10, sums=None):
        """Read the refinement history (host copy `sums` if given, taken after
        the stream completed); continue eagerly until rho <= tol."""
        torch.cuda.current_stream().synchronize()
        self.ctx.sync_status()
        res = SimResult(self.case.mesh_id)
        sums = self.sums.cpu().tolist() if sums is None else sums
        res.rho_hist = [self._rho(s) for s in sums]
        res.iters = [g.read()["iters"] for g in self.gm]
        rho = res.rho_hist[-1]
        while not rho <= self.tol and res.eager_steps < max_eager:
            if not math.isfinite(rho):
                raise api.IedgError(-4, f"mesh {self.case.mesh_id}: refinement residual is not finite")
            # the last residual left rF, rG in place: one more correction
            crtol = max(1e-7, min(0.1, 0.1 * self.tol / rho))
            p = self.prec
            api.condense_rhs(self.ctx, self.fac, self.rF, prec=p, w=self.wc, r=self.rc)
            api.assemble(self.ctx, self.mesh, r=self.rc, G=self.rG, prec=p, R=self.Rc)
            # restarted GMRES in the workspace of the first captured cycle
            gm = self.gm[0]
            _, info = api.gmres_solve(self.ctx, self.mesh, self.K, self.M, self.Rc, gm.steps, crtol,
                                      kprec=p, mprec=p, x=self.du, state=gm)
            api.backsolve_local(self.ctx, self.mesh, self.fac, self.du, prec=p, w=self.wc, z=self.dz)
            api.axpy(self.ctx, 1.0, self.du, self.uhat)
            api.axpy(self.ctx, 1.0, self.dz, self.z)
            self._enqueue_residual(self.n_refine)
            rho = self._rho(self.sums[self.n_refine].cpu().tolist())
            res.rho_hist.append(rho)
            res.iters.append(info["iters"])
            res.eager_steps += 1
        res.converged = rho <= self.tol
        return res

    def close(self):
        for g in self.gm:
            g.close()
        self.gm = []
        self.detach()
        self.mesh.close()


def _nnzb_estimate(hm):
    """Nonzero b x b blocks of K: sum over faces of the distinct faces that
    share an element with it."""
    import numpy as np
    ef = hm.elem_faces()
    nb = [set() for _ in range(hm.n_face)]
    for row in ef:
        for f in row:
            nb[f].update(int(g) for g in row)
    return int(sum(len(s) for s in nb))


class BatchGroup:
    """Meshes solved together: one persistent condensation launch over
    every mesh of a precision (all element sizes), then every mesh's trace
    solve; optionally captured in a graph."""

    def __init__(self, ctx, sims):
        self.ctx, self.sims = ctx, sims
        by_prec = {}
        for s in sims:
            by_prec.setdefault(s.prec, []).append(s)
        self.plans = [api.CondenseBatch(ctx, [s.condense_segment() for s in group], prec=prec)
                      for prec, group in sorted(by_prec.items())]
        self.graph = None

    def enqueue(self):
        for pl in self.plans:
            pl.run()
        for s in self.sims:
            s.enqueue_after_condense()

    def capture(self):
        """Capture enqueue() in a graph (after an eager run has set up every
        kernel's launch attributes)."""
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, capture_error_mode="thread_local"):
            self.enqueue()
        self.graph = g
        return g

    def run(self):
        if self.graph is not None:
            self.graph.replay()
        else:
            self.enqueue()

    def finish(self):
        return [s.finish() for s in self.sims]

    def close(self):
        for pl in self.plans:
            pl.close()
        self.graph = None


def plan_groups(cases, budget_bytes, prec=F32, restart=100, n_refine=1):
    """Greedy first-fit-decreasing packing of meshes into memory groups."""
    sized = sorted(((Simulation.footprint(c, prec, restart, n_refine), c) for c in cases),
                   key=lambda x: -x[0])
    groups = []
    for sz, c in sized:
        if sz > budget_bytes:
            raise ValueError(f"mesh {c.mesh_id} needs {sz / 1e9:.1f} GB > budget {budget_bytes / 1e9:.1f} GB")
        for g in groups:
            if g[0] + sz <= budget_bytes:
                g[0] += sz
                g[1].append(c)
                break
        else:
            groups.append([sz, [c]])
    return [sorted(g[1], key=lambda c: c.mesh_id) for g in groups]


def run_batch(ctx, workload, budget_bytes=160e9, prec=F32, use_graph=True, replays=1, n_refine=1,
              cases=None, log=None):
    """Solve every mesh of `workload` (batched form).  Returns a dict with
    per-mesh results and timings (generation excluded)."""
    from .autotune import apply_tuning
    apply_tuning(ctx)
    cases = workload.meshes if cases is None else cases
    groups = plan_groups(cases, budget_bytes, prec, workload.restart, n_refine)
    results, t_solve, t_min, t_med, elements = [], 0.0, 0.0, 0.0, 0
    for gi, gcases in enumerate(groups):
        sims = [Simulation(ctx, c, workload.seed, prec=prec, restart=workload.restart, n_refine=n_refine,
                           tol=workload.rtol) for c in gcases]
        for s in sims:
            s.generate()
        grp = BatchGroup(ctx, sims)
        grp.enqueue()           # eager run: sets launch attributes, checks the path
        torch.cuda.synchronize()
        ctx.sync_status()
        if use_graph:
            grp.capture()
        times = []
        for _ in range(replays):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            grp.run()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        t_fin0 = time.perf_counter()
        res = grp.finish()
        t_fin = time.perf_counter() - t_fin0
        # the mean replay (with the host's read of the residuals) is the
        # reported time; the fastest and the median replay are kept beside it
        t_group = sum(times) / len(times) + t_fin
        t_solve += t_group
        t_min += min(times) + t_fin
        t_med += sorted(times)[len(times) // 2] + t_fin
        elements += sum(s.E for s in sims)
        results.extend(res)
        if log:
            log(f"group {gi}: meshes {[c.mesh_id for c in gcases]} elements {sum(s.E for s in sims)} "
                f"time {t_group * 1e3:.1f} ms (replays {[round(t * 1e3, 1) for t in times]})")
        grp.close()
        for s in sims:
            s.close()
        del grp, sims
        torch.cuda.empty_cache()
    results.sort(key=lambda r: r.mesh_id)
    return {"results": results, "seconds": t_solve, "seconds_min": t_min, "seconds_median": t_med,
            "elements": elements, "groups": len(groups)}
