"""Thin Python binding of libiedg: argument marshalling only.

Every array is a torch tensor on the GPU (device memory and streams are the
only things torch provides here); every step runs in the library's HIP
kernels.  Functions enqueue on torch's current stream.
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import F64, F32, BF16, CondenseSegment, GmresOpts, GmresInfo, MeshInfo, RasInfo

PREC_DTYPE = {F64: torch.float64, F32: torch.float32, BF16: torch.float32}


class IedgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_lib.STATUS.get(status, status)}: {msg}")
        self.status = status


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_dev(*ts):
    for t in ts:
        if t is not None:
            if not t.is_cuda:
                raise ValueError("tensor must be on the GPU")
            if not t.is_contiguous():
                raise ValueError("tensor must be contiguous")


class Context:
    def __init__(self, device=None):
        self.L = _lib.load()
        dev = torch.cuda.current_device() if device is None else device
        h = ctypes.c_void_p()
        st = self.L.iedg_create(ctypes.byref(h), dev)
        if st != 0:
            raise IedgError(st, "iedg_create failed")
        self.h = h

    def check(self, st):
        if st != 0:
            raise IedgError(st, self.L.iedg_last_error(self.h).decode())

    def sync_status(self):
        """Synchronise and raise if a kernel latched a device-side error."""
        idx = ctypes.c_int64(-1)
        st = self.L.iedg_sync_status(self.h, _stream(), ctypes.byref(idx))
        if st != 0:
            err = IedgError(st, self.L.iedg_last_error(self.h).decode())
            err.index = idx.value
            raise err

    def clear_status(self):
        """Synchronise and discard any latched device-side error."""
        idx = ctypes.c_int64(-1)
        self.L.iedg_sync_status(self.h, _stream(), ctypes.byref(idx))

    def close(self):
        if self.h:
            self.L.iedg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mesh:
    """Trace topology + BSR pattern + BILU(0) schedule (iedg_mesh).
    elem_faces [E][6]: face-private trace units (iedg_mesh_create); any other
    width S: element slots of unit_dofs each, e.g. the nodes of the IEDG
    numbering (iedg_mesh_create_slots; n_face counts the units)."""

    def __init__(self, ctx, elem_faces, n_face, face_dofs, ordering="colour", order=None, slots=False):
        self.ctx = ctx
        ef = np.ascontiguousarray(elem_faces, dtype=np.int32)
        code = {"colour": 0, "natural": 1, "given": 2}[ordering]
        ordp = None
        if order is not None:
            order = np.ascontiguousarray(order, dtype=np.int32)
            ordp = order.ctypes.data_as(ctypes.c_void_p)
        h = ctypes.c_void_p()
        if ef.shape[1] == 6 and not slots:
            ctx.check(ctx.L.iedg_mesh_create(ctx.h, ef.shape[0], int(n_face), int(face_dofs),
                                             ef.ctypes.data_as(ctypes.c_void_p), code, ordp,
                                             ctypes.byref(h)))
        else:
            ctx.check(ctx.L.iedg_mesh_create_slots(ctx.h, ef.shape[0], ef.shape[1], int(n_face), int(face_dofs),
                                                   ef.ctypes.data_as(ctypes.c_void_p), code, ordp,
                                                   ctypes.byref(h)))
        self.h = h
        info = MeshInfo()
        ctx.check(ctx.L.iedg_mesh_query(h, ctypes.byref(info), None, None, None, None))
        self.info = info
        self.n_elem, self.n_face, self.b = info.n_elem, info.n_face, info.face_dofs
        self.slots = ef.shape[1]
        self.t = self.slots * self.b
        self.n_trace, self.nnzb, self.n_levels = info.n_trace, info.nnzb, info.n_levels

    def query(self):
        o = np.empty(self.n_face, np.int32)
        lp = np.empty(self.n_levels + 1, np.int32)
        rp = np.empty(self.n_face + 1, np.int32)
        cf = np.empty(self.nnzb, np.int32)
        ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        self.ctx.check(self.ctx.L.iedg_mesh_query(self.h, None, ptr(o), ptr(lp), ptr(rp), ptr(cf)))
        return {"order": o, "level_ptr": lp, "row_ptr": rp, "col_face": cf}

    def close(self):
        if self.h:
            self.ctx.L.iedg_mesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def condense(ctx, A, B, C, D, F=None, prec=F64, out=None):
    """a1: returns dict LU, perm, U12, L21, w, Ke, r (see iedg_condense)."""
    _check_dev(A, B, C, D, F)
    E, n, _ = A.shape
    t = B.shape[2]
    dt = PREC_DTYPE[prec]
    o = out if out is not None else {}
    dev = A.device
    def need(key, shape, dtype):
        if key not in o:
            o[key] = torch.empty(shape, dtype=dtype, device=dev)
        return o[key]
    LU = need("LU", (E, n, n), dt)
    perm = need("perm", (E, n), torch.int32)
    U12 = need("U12", (E, n, t), dt)
    L21 = need("L21", (E, t, n), dt)
    Ke = need("Ke", (E, t, t), dt)
    w = need("w", (E, n), torch.float64) if F is not None else None
    r = need("r", (E, t), torch.float64) if F is not None else None
    ctx.check(ctx.L.iedg_condense(ctx.h, E, n, t, prec, _p(A), _p(B), _p(C), _p(D), _p(F),
                                  _p(LU), _p(perm), _p(U12), _p(L21), _p(w), _p(Ke), _p(r), _stream()))
    return o


def alloc_condense_out(E, n, t, prec, device, with_rhs=True):
    """Output buffers of iedg_condense for E elements."""
    dt = PREC_DTYPE[prec]
    o = {"LU": torch.empty((E, n, n), dtype=dt, device=device),
         "perm": torch.empty((E, n), dtype=torch.int32, device=device),
         "U12": torch.empty((E, n, t), dtype=dt, device=device),
         "L21": torch.empty((E, t, n), dtype=dt, device=device),
         "Ke": torch.empty((E, t, t), dtype=dt, device=device)}
    if with_rhs:
        o["w"] = torch.empty((E, n), dtype=torch.float64, device=device)
        o["r"] = torch.empty((E, t), dtype=torch.float64, device=device)
    return o


class CondenseBatch:
    """Plan for one persistent condensation launch over several segments
    (meshes), of one element size or of several (iedg_batch_create_sized).
    `segments` is a list of (inputs, outputs) dicts: inputs A, B, C, D, F (F
    may be None), outputs as from alloc_condense_out.  Tensors must outlive
    the plan."""

    def __init__(self, ctx, segments, prec=F64):
        self.ctx = ctx
        self._keep = segments
        k = len(segments)
        arr = (CondenseSegment * k)()
        ns = (ctypes.c_int32 * k)()
        ts = (ctypes.c_int32 * k)()
        for i, (inp, out) in enumerate(segments):
            _check_dev(inp["A"], inp["B"], inp["C"], inp["D"], inp.get("F"))
            E, ns[i], _ = inp["A"].shape
            ts[i] = inp["B"].shape[2]
            a = arr[i]
            a.n_elem = E
            a.A, a.B, a.C, a.D = (inp[key].data_ptr() for key in "ABCD")
            a.F = inp["F"].data_ptr() if inp.get("F") is not None else None
            a.LU, a.perm, a.U12, a.L21, a.Ke = (out[key].data_ptr() for key in ("LU", "perm", "U12", "L21", "Ke"))
            a.w = out["w"].data_ptr() if "w" in out else None
            a.r = out["r"].data_ptr() if "r" in out else None
        h = ctypes.c_void_p()
        ctx.check(ctx.L.iedg_batch_create_sized(ctx.h, k, arr, ctypes.cast(ns, ctypes.c_void_p),
                                                ctypes.cast(ts, ctypes.c_void_p), prec, ctypes.byref(h)))
        self.h, self.prec = h, prec
        self.sizes = sorted({(ns[i], ts[i]) for i in range(k)}, reverse=True)

    def run(self):
        self.ctx.check(self.ctx.L.iedg_condense_batched(self.ctx.h, self.h, _stream()))

    def close(self):
        if self.h:
            self.ctx.L.iedg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def set_leaf_width(ctx, n_local, leaf_width, prec=F32):
    """Sub-panel width (8 or 16) of the condensation kernel for (prec, n)."""
    ctx.check(ctx.L.iedg_set_leaf_width(ctx.h, int(prec), int(n_local), int(leaf_width)))


def set_panel_width(ctx, n_local, panel_width, prec=F32):
    """Panel width (64, or 128 in FP32 storage) of the condensation for (prec, n)."""
    ctx.check(ctx.L.iedg_set_panel_width(ctx.h, int(prec), int(n_local), int(panel_width)))


class GmresState:
    """GMRES workspace of one mesh (iedg_gmres_state_*), allocated once.
    gmres_solve(..., state=) runs restarted GMRES in it; enqueue() runs one
    device-driven cycle with no host synchronisation (it can be captured in a
    graph) and read() returns its outcome after the stream has completed."""

    def __init__(self, ctx, mesh, steps):
        self.ctx, self.mesh = ctx, mesh
        h = ctypes.c_void_p()
        ctx.check(ctx.L.iedg_gmres_state_create(ctx.h, mesh.h, int(steps), ctypes.byref(h)))
        self.h, self.steps = h, steps

    def enqueue(self, Kbsr, Mbsr, R, x, rtol, inner_factor=0.1, kprec=F64, mprec=F64):
        _check_dev(Kbsr, Mbsr, R, x)
        self.ctx.check(self.ctx.L.iedg_gmres_enqueue(self.ctx.h, self.mesh.h, self.h, kprec, _p(Kbsr), mprec,
                                                     _p(Mbsr), _p(R), _p(x), float(rtol), float(inner_factor),
                                                     _stream()))

    def set_ras(self, ras):
        """Precondition with the RAS `ras` (its factors are then the M
        argument); None restores BILU(0) of the mesh."""
        self.ctx.check(self.ctx.L.iedg_gmres_state_set_ras(self.ctx.h, self.h, None if ras is None else ras.h))
        self._ras = ras

    def read(self):
        info = GmresInfo()
        self.ctx.check(self.ctx.L.iedg_gmres_state_read(self.ctx.h, self.h, ctypes.byref(info)))
        return {"iters": info.iters, "converged": bool(info.converged), "rel_resid": info.rel_resid}

    def close(self):
        if self.h:
            self.ctx.L.iedg_gmres_state_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def condense_rhs(ctx, fac, F, prec=F64, w=None, r=None):
    LU, perm, L21 = fac["LU"], fac["perm"], fac["L21"]
    E, n, _ = LU.shape
    t = L21.shape[1]
    w = torch.empty((E, n), dtype=torch.float64, device=F.device) if w is None else w
    r = torch.empty((E, t), dtype=torch.float64, device=F.device) if r is None else r
    ctx.check(ctx.L.iedg_condense_rhs(ctx.h, E, n, t, prec, _p(LU), _p(perm), _p(L21), _p(F),
                                      _p(w), _p(r), _stream()))
    return w, r


def assemble(ctx, mesh, Ke=None, r=None, G=None, prec=F64, Kbsr=None, R=None):
    if Ke is not None and Kbsr is None:
        Kbsr = torch.empty((mesh.nnzb, mesh.b, mesh.b), dtype=PREC_DTYPE[prec], device=Ke.device)
    dev = (Ke if Ke is not None else (r if r is not None else G)).device
    if (r is not None or G is not None) and R is None:
        R = torch.empty(mesh.n_trace, dtype=torch.float64, device=dev)
    ctx.check(ctx.L.iedg_assemble(ctx.h, mesh.h, prec, _p(Ke), _p(r), _p(G), _p(Kbsr), _p(R), _stream()))
    return Kbsr, R


def factor_ilu0(ctx, mesh, Kbsr, prec=F64, Mbsr=None):
    Mbsr = torch.empty_like(Kbsr) if Mbsr is None else Mbsr
    ctx.check(ctx.L.iedg_factor_ilu0(ctx.h, mesh.h, prec, _p(Kbsr), _p(Mbsr), _stream()))
    return Mbsr


class Ras:
    """Restricted additive Schwarz preconditioner over a face partition
    (iedg_ras_*): part[f] = subdomain of face f, `delta` overlap layers."""

    def __init__(self, ctx, mesh, part, delta):
        self.ctx, self.mesh = ctx, mesh
        part = np.ascontiguousarray(part, dtype=np.int32)
        n_sub = int(part.max()) + 1
        h = ctypes.c_void_p()
        ctx.check(ctx.L.iedg_ras_create(ctx.h, mesh.h, n_sub, part.ctypes.data_as(ctypes.c_void_p), int(delta),
                                        ctypes.byref(h)))
        self.h = h
        info = RasInfo()
        ctx.check(ctx.L.iedg_ras_query(h, ctypes.byref(info)))
        self.n_sub, self.delta = info.n_sub, info.delta
        self.n_local_rows, self.nnzb, self.n_levels = info.n_local_rows, info.nnzb, info.n_levels

    def factor(self, Kbsr, prec=F64, Mloc=None):
        _check_dev(Kbsr)
        if Mloc is None:
            Mloc = torch.empty((self.nnzb, self.mesh.b, self.mesh.b), dtype=PREC_DTYPE[prec], device=Kbsr.device)
        self.ctx.check(self.ctx.L.iedg_ras_factor(self.ctx.h, self.h, prec, _p(Kbsr), _p(Mloc), _stream()))
        return Mloc

    def apply(self, Mloc, x, prec=F64, y=None):
        y = torch.empty_like(x) if y is None else y
        self.ctx.check(self.ctx.L.iedg_ras_apply(self.ctx.h, self.h, prec, _p(Mloc), _p(x), _p(y), _stream()))
        return y

    def close(self):
        if self.h:
            self.ctx.L.iedg_ras_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mdf_order(ctx, mesh, Kbsr, prec=F64):
    """Minimum discarded fill order of the faces (iedg_mdf_order), host int32
    array; pass it to Mesh(..., ordering="given", order=...)."""
    _check_dev(Kbsr)
    order = np.empty(mesh.n_face, np.int32)
    ctx.check(ctx.L.iedg_mdf_order(ctx.h, mesh.h, prec, _p(Kbsr), order.ctypes.data_as(ctypes.c_void_p), _stream()))
    return order


def gmres_solve(ctx, mesh, Kbsr, Mbsr, R, restart, rtol, max_iters=10000, inner_factor=0.1,
                kprec=F64, mprec=F64, precond=True, x=None, raise_on_fail=True, state=None):
    """GMRES(restart) in the workspace of `state` (a GmresState of this mesh
    with at least `restart` steps); without one, a state is created for this
    call and freed after it."""
    x = torch.empty_like(R) if x is None else x
    own = state is None
    if own:
        state = GmresState(ctx, mesh, restart)
    try:
        opts = GmresOpts(restart, max_iters, rtol, inner_factor, 1 if precond else 0)
        info = GmresInfo()
        st = ctx.L.iedg_gmres_solve(ctx.h, mesh.h, state.h, kprec, _p(Kbsr), mprec,
                                    _p(Mbsr) if precond else None, _p(R), _p(x), ctypes.byref(opts),
                                    ctypes.byref(info), _stream())
    finally:
        if own:
            state.close()
    res = {"iters": info.iters, "cycles": info.cycles, "converged": bool(info.converged),
           "rel_resid": info.rel_resid, "status": st}
    if st != 0 and (raise_on_fail or st != -3):
        ctx.check(st)
    return x, res


def spmv(ctx, mesh, Kbsr, x, prec=F64, y=None):
    y = torch.empty_like(x) if y is None else y
    ctx.check(ctx.L.iedg_spmv(ctx.h, mesh.h, prec, _p(Kbsr), _p(x), _p(y), _stream()))
    return y


def ilu0_apply(ctx, mesh, Mbsr, x, prec=F64, y=None):
    y = torch.empty_like(x) if y is None else y
    ctx.check(ctx.L.iedg_ilu0_apply(ctx.h, mesh.h, prec, _p(Mbsr), _p(x), _p(y), _stream()))
    return y


def backsolve_local(ctx, mesh, fac, uhat, prec=F64, w=None, z=None):
    LU, U12 = fac["LU"], fac["U12"]
    w = fac["w"] if w is None else w
    E, n, _ = LU.shape
    z = torch.empty((E, n), dtype=torch.float64, device=uhat.device) if z is None else z
    ctx.check(ctx.L.iedg_backsolve_local(ctx.h, mesh.h, n, prec, _p(LU), _p(fac["perm"]), _p(U12), _p(w),
                                         _p(uhat), _p(z), _stream()))
    return z


def residual_full(ctx, mesh, A, B, C, D, F, G, z, uhat, rF=None, rG=None, sums=None):
    E, n, _ = A.shape
    rF = torch.empty((E, n), dtype=torch.float64, device=A.device) if rF is None else rF
    rG = torch.empty_like(G) if rG is None else rG
    sums = torch.empty(4, dtype=torch.float64, device=A.device) if sums is None else sums
    ctx.check(ctx.L.iedg_residual_full(ctx.h, mesh.h, n, _p(A), _p(B), _p(C), _p(D), _p(F), _p(G),
                                       _p(z), _p(uhat), _p(rF), _p(rG), _p(sums), _stream()))
    return rF, rG, sums


def axpy(ctx, alpha, x, y):
    ctx.check(ctx.L.iedg_axpy(ctx.h, x.numel(), float(alpha), _p(x), _p(y), _stream()))
    return y


def probe_mfma(ctx, prec, n_wg=2048, iters=2048, reps=3, sink=None):
    """Measured MFMA ceiling for `prec` (iedg_probe_mfma): the best of `reps`
    launches timed with events on the current stream.  Returns (TFLOP/s,
    sink) -- sink holds each thread's accumulator sum, 32 K iters."""
    sink = torch.empty(n_wg * 512, dtype=torch.float64, device="cuda") if sink is None else sink
    flops = ctypes.c_double()
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.check(ctx.L.iedg_probe_mfma(ctx.h, int(prec), n_wg, iters, _p(sink), ctypes.byref(flops), _stream()))
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    return flops.value / (best * 1e-3) / 1e12, sink


def probe_triad(ctx, n=1 << 28, s=3.0, reps=5, arrays=None):
    """Measured HBM ceiling (iedg_probe_triad, a = b + s c over n doubles,
    24 n bytes): the best of `reps` launches.  Returns (GB/s, (a, b, c))."""
    if arrays is None:
        b = torch.ones(n, dtype=torch.float64, device="cuda")
        c = torch.full((n,), 0.5, dtype=torch.float64, device="cuda")
        a = torch.empty_like(b)
    else:
        a, b, c = arrays
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.check(ctx.L.iedg_probe_triad(ctx.h, n, _p(b), _p(c), float(s), _p(a), _stream()))
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    return 24.0 * n / (best * 1e-3) / 1e9, (a, b, c)


class MinResGuess:
    """Minimal-residual Newton initial guess (iedg_mr_*, section 2.2.1,
    eq. MinRes2) for one mesh and element size, workspace for up to s_max
    previous solutions allocated once."""

    def __init__(self, ctx, mesh, n_local, s_max):
        self.ctx, self.mesh, self.n, self.s_max = ctx, mesh, int(n_local), int(s_max)
        h = ctypes.c_void_p()
        ctx.check(ctx.L.iedg_mr_create(ctx.h, mesh.h, self.n, self.s_max, ctypes.byref(h)))
        self.h = h

    def residual(self, blocks, G, eps, Z, U, beta, R=None, sums=None):
        """R(point_k) for the points beta [m][s] (host array): returns R [m][E n + N_t], sums [m]."""
        beta = np.ascontiguousarray(beta, dtype=np.float64)
        m, s = beta.shape
        A, B, C, D, F = (blocks[k] for k in "ABCDF")
        _check_dev(A, B, C, D, F, G, Z, U)
        L = Z.shape[1] * Z.shape[2] + U.shape[1]
        R = torch.empty((m, L), dtype=torch.float64, device=A.device) if R is None else R
        sums = torch.empty(m, dtype=torch.float64, device=A.device) if sums is None else sums
        self.ctx.check(self.ctx.L.iedg_mr_residual(
            self.ctx.h, self.h, _p(A), _p(B), _p(C), _p(D), _p(F), _p(G), float(eps), s, _p(Z), _p(U), m,
            beta.ctypes.data_as(ctypes.c_void_p), _p(R), _p(sums), _stream()))
        return R, sums

    def guess(self, blocks, G, eps, Z, U, max_iters=20, lambda0=1e-3, fd_step=1e-7, tol=1e-10, ftol=1e-10, z0=None,
              u0=None):
        """alpha (numpy [s]), z0 [E][n], u0 [N_t] and info dict."""
        A, B, C, D, F = (blocks[k] for k in "ABCDF")
        _check_dev(A, B, C, D, F, G, Z, U)
        s = Z.shape[0]
        z0 = torch.empty(Z.shape[1:], dtype=torch.float64, device=A.device) if z0 is None else z0
        u0 = torch.empty(U.shape[1:], dtype=torch.float64, device=A.device) if u0 is None else u0
        alpha = np.zeros(s)
        opts = _lib.MrOpts(int(max_iters), float(lambda0), float(fd_step), float(tol), float(ftol))
        info = _lib.MrInfo()
        self.ctx.check(self.ctx.L.iedg_mr_guess(
            self.ctx.h, self.h, _p(A), _p(B), _p(C), _p(D), _p(F), _p(G), float(eps), s, _p(Z), _p(U),
            ctypes.byref(opts), alpha.ctypes.data_as(ctypes.c_void_p), _p(z0), _p(u0), ctypes.byref(info),
            _stream()))
        return alpha, z0, u0, {"iters": info.iters, "passes": info.passes, "obj0": info.obj0, "obj": info.obj}

    def close(self):
        if self.h:
            self.ctx.L.iedg_mr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
