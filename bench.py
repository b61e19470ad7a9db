#!/usr/bin/env python3
"""Newton-step solves/s of the IEDG trace solve on one MI355X.

Workload: one subdomain at the paper's shape -- a 16x16x8 structured hex mesh
with p = 3 (2,048 elements, n = 1,280 local dofs and t = 480 trace dofs per
element, 6,656 faces of 80 trace dofs, 532,480 trace unknowns), seeded
synthetic element blocks generated directly in HBM, ten right-hand sides.

A step is one full Newton-step linear solve: condensation of every element,
assembly of K and R, BILU(0), GMRES(100) and the element back-substitution,
plus FP64 iterative refinement for the mixed form.  Step k uses right-hand
side k mod 10.  Both forms are timed at the same tolerance: the relative
residual of the uncondensed system is <= 1e-8 (FP64 form: GMRES to 1e-8 on
K; mixed form: FP32 condensation / FP32 K and BILU(0), refined in FP64).

Prints one JSON line.

--workload batch: the 24-mesh uneven batch (mixed sizes and degrees), solved
by the batched form (persistent condensation launches, HIP graph replay per
memory group).  --workload serving: seeded Poisson requests against 64
simulations under a 200 GB residency budget (continuous batching over HIP
streams), reporting solves/s with p50/p99 latency.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0


# the sources of the FP32 condensation kernel (HBM counters are reported only
# while these are unchanged since the counters were taken)
CONDENSE_SOURCES = ["paper_1605_01020_amd/csrc/condense_kernel.h", "paper_1605_01020_amd/csrc/condense.h",
                    "paper_1605_01020_amd/csrc/condense_f32.hip", "paper_1605_01020_amd/csrc/condense_f32_single.hip",
                    "paper_1605_01020_amd/csrc/common.h",
                    "paper_1605_01020_amd/tuning.json"]


def condense_flops(n, t):
    # LU of A, U12 = L^{-1} P B, L21 = C U^{-1}, Schur product L21 U12
    return (2.0 / 3.0) * n ** 3 + 2.0 * n * n * t + 2.0 * n * t * t


def cpu_baseline(seed, restart):
    """The FP64 oracle on a bounded sample, scaled to one full step."""
    import numpy as np
    import oracle
    from synth import StructuredHexMesh, ElementSpec, element_inputs, trace_rhs
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count()
    from oracle.assembly import matvec
    sub = StructuredHexMesh(4, 2, 2)
    spec = ElementSpec(3)
    blocks = [element_inputs(spec, seed, 0, e) for e in range(sub.n_elem)]
    G = trace_rhs(spec, seed, 0, sub.n_face)
    tm = oracle.TraceMesh(sub.elem_faces(), sub.n_face, spec.b)
    runs = []
    for _ in range(3):
        t0 = time.perf_counter()
        Ks, rs = oracle.condense_all(blocks)
        t1 = time.perf_counter()
        K, R = oracle.assemble(tm, Ks, rs, G)
        fac = oracle.bilu0(tm, K, oracle.greedy_colour_order(tm))
        uhat, info = oracle.gmres(lambda v: matvec(tm, K, v), lambda v: oracle.bilu0_apply(tm, fac, v), R,
                                  restart, 1e-8)
        t2 = time.perf_counter()
        oracle.backsolve_all(tm, blocks, uhat)
        t3 = time.perf_counter()
        runs.append((t1 - t0, t2 - t1, t3 - t2))
    med = [float(np.median([r[i] for r in runs])) for i in range(3)]
    full = StructuredHexMesh(16, 16, 8)
    per_elem = (med[0] + med[2]) / sub.n_elem
    per_face = med[1] / sub.n_face
    step_s = per_elem * full.n_elem + per_face * full.n_face
    work = sum(sum(r) for r in runs)
    cpu_model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": 1.0 / step_s, "unit": "Newton-step solves/s", "cores": int(threads), "kind": "oracle",
            "cpu_model": cpu_model, "nproc": os.cpu_count(), "blas_threads": int(threads),
            "sample": (f"oracle FP64 solve of a 4x2x2 p=3 mesh with the same distributions ({sub.n_elem} "
                       f"elements, {sub.n_face} faces, {info['iters']} GMRES iterations), median of 3; element "
                       f"phases scaled by {full.n_elem}/{sub.n_elem}, trace phases by {full.n_face}/{sub.n_face}; "
                       f"{work:.1f} s of CPU work"),
            "condense_elems_per_s": sub.n_elem / med[0]}


def measured_traffic(kernel_sources, profile):
    """HBM bytes per launch from a rocprofv3 counter summary, or None when the
    kernel source (or its tuning table) changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for src in kernel_sources:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#", " ")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("source-sha256") != h.hexdigest():
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def batch_form(ctx, prec, args, replays=2):
    """The 24-mesh uneven batch in one precision form (F32: FP32 condensation
    and trace system with FP64 refinement; F64: plain FP64).  Time: mean of
    the graph replays per memory group (generation excluded)."""
    import torch
    from paper_1605_01020_amd.batch import run_batch
    from synth.matrices import workload
    wl = workload(3)
    out = run_batch(ctx, wl, budget_bytes=args.budget_gb * 1e9, prec=prec, replays=replays, log=_log)
    res = out["results"]
    E = sum(m.mesh.n_elem for m in wl.meshes)
    torch.cuda.empty_cache()
    return {"solves_per_s": len(res) / out["seconds"], "seconds": out["seconds"],
            "seconds_min_replay": out["seconds_min"], "seconds_median_replay": out["seconds_median"],
            "elements_per_s": E / out["seconds"], "groups": out["groups"],
            "max_rho_full": max(r.rho_hist[-1] for r in res), "all_converged": all(r.converged for r in res),
            "eager_steps": sum(r.eager_steps for r in res)}


def bench_batch(args):
    """Batched form over the 24-mesh uneven batch; a step is one pass over
    every mesh (generation of the inputs excluded from the timed region)."""
    import torch
    from paper_1605_01020_amd import api, F32, F64
    from paper_1605_01020_amd.autotune import apply_tuning
    from synth.matrices import workload
    wl = workload(3)
    torch.cuda.set_device(0)
    ctx = api.Context(0)
    apply_tuning(ctx)
    E = sum(m.mesh.n_elem for m in wl.meshes)
    flops = sum(condense_flops(m.spec.n, m.spec.t) * m.mesh.n_elem for m in wl.meshes)
    forms = {"f32": batch_form(ctx, F32, args, max(1, args.steps)), "f64": batch_form(ctx, F64, args, max(1, args.steps))}
    r = forms["f32"]
    line = {
        "metric": "Newton-step solves/s at relative residual 1e-8, batched form (24 uneven meshes)",
        "value": r["solves_per_s"], "unit": "Newton-step solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": r["seconds"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic (seeded Philox element blocks generated in HBM per memory group)",
        "config": {"workload": f"24 meshes from {{4^3, 6^3, 8x8x4, 12x12x6}} x p in {{2,3,4}}, E={E}, "
                               f"condensation {flops:.3e} flop, GMRES(100)+BILU(0), tol 1e-8",
                   "budget_gb": args.budget_gb},
        "forms": forms,
        "speedup_mixed_vs_fp64": forms["f32"]["solves_per_s"] / forms["f64"]["solves_per_s"],
        "condense_tflops_equiv": flops / r["seconds"] / 1e12,
    }
    print(json.dumps(line), flush=True)


def serving_sweep(ctx, fracs, n_warm, n_meas, slots, budget_gb, n_cap=None, log=_log):
    """The serving form over the 64 simulations of the uneven distribution:
    closed-loop capacity first (every request available at once, after a
    warm-up that fills the residency cache), then Poisson arrivals at each
    fraction of that capacity; latency and hit rate over the measured
    requests only (the first n_warm of each stream warm the cache)."""
    import numpy as np
    from paper_1605_01020_amd import F32
    from paper_1605_01020_amd.serve import Server, poisson_requests, summarize
    from synth.matrices import workload
    wl = workload(4)
    n_cap = n_meas if n_cap is None else n_cap
    srv = Server(ctx, wl.meshes, wl.seed, budget_bytes=budget_gb * 1e9, n_slots=slots, prec=F32,
                 restart=wl.restart, tol=wl.rtol)
    out = {"simulations": len(wl.meshes), "slots": slots, "budget_gb": budget_gb,
           "static_gb": srv.static_bytes / 1e9}
    def progress(k, total):
        log(f"  {k}/{total} requests done")

    reqs = poisson_requests(wl.seed, n_warm + n_cap, 1e6, len(wl.meshes))
    srv.run(reqs[:n_warm], real_time=False, progress=progress)
    t0 = time.perf_counter()
    done = srv.run(reqs[n_warm:], real_time=False, progress=progress)
    cap = len(done) / (time.perf_counter() - t0)
    out["capacity_solves_per_s"] = cap
    out["capacity_hit_rate"] = sum(1 for r in done if r.hit) / len(done)
    log(f"serving capacity {cap:.2f} solves/s over {len(done)} requests (hit rate {out['capacity_hit_rate']:.2f})")
    out["load"] = {}
    for i, frac in enumerate(fracs):
        rate = frac * cap
        reqs = poisson_requests(wl.seed + 1 + i, n_warm + n_meas, rate, len(wl.meshes))
        t0 = time.perf_counter()
        done = srv.run(reqs, real_time=True, progress=progress)
        elapsed = time.perf_counter() - t0
        meas = [r for r in done if r.rid >= n_warm]
        span = max(r.done for r in meas) - min(r.arrival for r in meas)
        s = summarize(meas, span)
        s["rate_per_s"] = rate
        out["load"][f"{frac:.1f}"] = s
        log(f"load {frac:.1f} x capacity ({rate:.2f}/s): {s['solves_per_s']:.2f} solves/s, p50 {s['p50_ms']:.0f} ms, "
            f"p99 {s['p99_ms']:.0f} ms, hit rate {s['hit_rate']:.2f} ({elapsed:.0f} s)")
    out["stats"] = dict(srv.stats)
    srv.close()
    return out


def bench_serving(args):
    import torch
    from paper_1605_01020_amd import api
    from paper_1605_01020_amd.autotune import apply_tuning
    torch.cuda.set_device(0)
    ctx = api.Context(0)
    apply_tuning(ctx)
    fracs = [float(f) for f in args.loads.split(",")]
    res = serving_sweep(ctx, fracs, args.serve_warmup, args.requests, args.slots, args.budget_gb,
                        n_cap=args.capacity_requests)
    head = res["load"][f"{fracs[len(fracs) // 2]:.1f}"]
    line = {
        "metric": "Newton-step solves/s at relative residual 1e-8 with p50/p99 latency, serving form",
        "value": head["solves_per_s"], "unit": "Newton-step solves/s", "n_gpus": 1, "steps": args.requests,
        "warmup": args.serve_warmup, "ms_per_step": 1e3 / head["solves_per_s"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic (seeded Poisson arrivals and Philox matrices)",
        "config": {"workload": f"{res['simulations']} simulations from the uneven batch distribution, Poisson "
                               f"arrivals at {fracs} x measured capacity ({args.capacity_requests} closed-loop "
                               f"requests), {args.serve_warmup} warm-up + "
                               f"{args.requests} measured requests per load, budget {args.budget_gb} GB, "
                               f"{args.slots} stream slots"},
        "serving": res,
    }
    print(json.dumps(line), flush=True)


def _ms(fn, reps=1):
    """Average milliseconds of fn() on the current stream (HIP events)."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def extra_fp64_tight(ctx, mesh, n, mats, Fs, Gs, restart, rtol=1e-10, steps=3):
    """The plain FP64 form at the workload's own tolerance (1e-10 on K)."""
    import torch
    from paper_1605_01020_amd.solver import NewtonStepSolver
    A, B, C, D = mats
    solver = NewtonStepSolver(ctx, mesh, n, restart=restart)
    solver.solve_fp64(A, B, C, D, Fs[0], Gs[0], rtol=rtol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    for k in range(steps):
        _, _, info = solver.solve_fp64(A, B, C, D, Fs[k % len(Fs)], Gs[k % len(Gs)], rtol=rtol)
        iters.append(info["iters"])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    return {"solves_per_s": 1e3 / ms, "ms_per_step": ms, "rtol": rtol, "gmres_iters": iters}


def extra_rhs_solves(ctx, mesh, n, mats, Fs, Gs, restart):
    """Right-hand-side-only solves with retained factors: every right-hand
    side of the sequence after one factorisation (FP64 at 1e-10 and 1e-8;
    mixed FP32 with FP64 refinement at 1e-8)."""
    import torch
    from paper_1605_01020_amd import api, F64, F32
    from paper_1605_01020_amd.solver import NewtonStepSolver
    A, B, C, D = mats
    out = {}
    for name, prec, tol in (("fp64_1e-10", F64, 1e-10), ("fp64_1e-8", F64, 1e-8), ("mixed_f32_1e-8", F32, 1e-8)):
        solver = NewtonStepSolver(ctx, mesh, n, restart=restart)
        solver.factor(A, B, C, D, None, prec=prec)
        torch.cuda.synchronize()
        iters, rhos = [], []
        t0 = time.perf_counter()
        for F, G in zip(Fs, Gs):
            if prec == F64:
                z, u, info = solver.solve_rhs_fp64(F, G, tol)
            else:
                z, u, info = solver.solve_rhs_mixed(A, B, C, D, F, G, tol=tol)
                rhos.append(info["rho_full"])
            iters.append(info["iters"])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / len(Fs)
        out[name] = {"rhs_solves_per_s": 1e3 / ms, "ms_per_rhs": ms, "gmres_iters": iters}
        if rhos:
            out[name]["max_rho_full"] = max(rhos)
        del solver
        torch.cuda.empty_cache()
    return out


def extra_mr_guess(ctx, mesh, n, mats, F, G, restart, svals=(3, 6), eps=0.05):
    """Minimal-residual Newton initial guess (eq. MinRes2) over s previous
    solutions x_j = (1 + 0.1 (j + 1)) x + 0.01 N(0, 1) around the FP64
    Newton-step solution x, on the cubic residual with eps: time, passes
    over the element blocks and the objective reduction."""
    import numpy as np
    import torch
    from paper_1605_01020_amd import api
    from paper_1605_01020_amd.solver import NewtonStepSolver
    A, B, C, D = mats
    solver = NewtonStepSolver(ctx, mesh, n, restart=restart)
    z, u, _ = solver.solve_fp64(A, B, C, D, F, G, rtol=1e-10)
    del solver
    blocks = {"A": A, "B": B, "C": C, "D": D, "F": F}
    block_bytes = 8 * (A.numel() + B.numel() + C.numel() + D.numel())
    out = {}
    for s in svals:
        g = torch.Generator(device="cuda").manual_seed(s)
        Z = torch.stack([(1.0 + 0.1 * (j + 1)) * z + 0.01 * torch.randn(z.shape, generator=g, device="cuda",
                                                                        dtype=torch.float64) for j in range(s)])
        U = torch.stack([(1.0 + 0.1 * (j + 1)) * u + 0.01 * torch.randn(u.shape, generator=g, device="cuda",
                                                                        dtype=torch.float64) for j in range(s)])
        mr = api.MinResGuess(ctx, mesh, n, s)
        mr.guess(blocks, G, eps, Z, U)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        alpha, z0, u0, info = mr.guess(blocks, G, eps, Z, U)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        pass_ms = _ms(lambda: mr.residual(blocks, G, eps, Z, U, np.tile(alpha, (s + 1, 1))), 3)
        out[f"s{s}"] = {"ms": ms, "passes": info["passes"], "lm_steps": info["iters"],
                        "pass_ms": pass_ms, "pass_block_TBps": block_bytes / (pass_ms * 1e-3) / 1e12,
                        "obj_ratio": info["obj"] / info["obj0"], "alpha": [float(a) for a in alpha], "eps": eps}
        mr.close()
        del Z, U
        torch.cuda.empty_cache()
    return out


def extra_iedg(ctx, hmesh, spec, mats, F, restart, wl_seed):
    """The same element matrices assembled on the IEDG trace numbering
    (nodes shared along interior faces, 5 x 5 node blocks): system size,
    levels, and the FP64 (1e-8) and FP32-mixed (1e-8) Newton-step solves
    with their phase times.  G is the IEDG-sized draw of the same stream."""
    import numpy as np
    import torch
    import synth.device as sd
    from paper_1605_01020_amd import api, F32
    from paper_1605_01020_amd.solver import NewtonStepSolver, StepTimer
    A, B, C, D = mats
    en, n_nodes = hmesh.iedg_trace_nodes(spec.p)
    t0 = time.perf_counter()
    mesh = api.Mesh(ctx, en, n_nodes, 5)
    setup_s = time.perf_counter() - t0
    G = sd.gen_trace_rhs(spec, wl_seed, 0, hmesh.n_face, count=n_nodes * 5)
    out = {"n_nodes": n_nodes, "n_trace": int(mesh.n_trace), "nnzb": int(mesh.nnzb), "block": 5,
           "levels": int(mesh.n_levels), "mesh_setup_s": setup_s}
    for name, mixed in (("fp64_1e-8", False), ("mixed_f32_1e-8", True)):
        solver = NewtonStepSolver(ctx, mesh, spec.n, restart=restart)
        run = (lambda tm: solver.solve_mixed(A, B, C, D, F, G, tol=1e-8, prec=F32, timer=tm)) if mixed else \
              (lambda tm: solver.solve_fp64(A, B, C, D, F, G, rtol=1e-8, timer=tm))
        run(None)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        z, u, _ = run(None)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        z, u, info = run(StepTimer(True))
        _, _, sums = api.residual_full(ctx, mesh, A, B, C, D, F, G, z, u)
        sh = sums.cpu().numpy()
        out[name] = {"solves_per_s": 1e3 / ms, "ms_per_step": ms, "gmres_iters": info["iters"],
                     "rho_full": float(np.sqrt((sh[0] + sh[1]) / (sh[2] + sh[3]))),
                     "phases_ms": info.get("phases_ms")}
        del solver
        torch.cuda.empty_cache()
    mesh.close()
    return out


def extra_orderings(ctx, hmesh, spec, mats, F, G, restart, rtol=1e-10):
    """BILU(0) under the natural, colour and minimum discarded fill orders
    (FP64): levels, factorisation and application time, GMRES iterations."""
    import torch
    from paper_1605_01020_amd import api, F64
    A, B, C, D = mats
    fac = api.condense(ctx, A, B, C, D, F, prec=F64)
    out = {}
    meshes = {}
    for name in ("natural", "colour", "mdf"):
        if name == "mdf":
            base = meshes["colour"]
            Kc, _ = api.assemble(ctx, base, Ke=fac["Ke"], prec=F64)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            order = api.mdf_order(ctx, base, Kc, prec=F64)
            t_mdf = time.perf_counter() - t0
            del Kc
            mesh = api.Mesh(ctx, hmesh.elem_faces(), hmesh.n_face, spec.b, ordering="given", order=order)
        else:
            mesh = api.Mesh(ctx, hmesh.elem_faces(), hmesh.n_face, spec.b, ordering=name)
        meshes[name] = mesh
        K, R = api.assemble(ctx, mesh, Ke=fac["Ke"], r=fac["r"], G=G, prec=F64)
        M = torch.empty_like(K)
        api.factor_ilu0(ctx, mesh, K, prec=F64, Mbsr=M)
        t_fac = _ms(lambda: api.factor_ilu0(ctx, mesh, K, prec=F64, Mbsr=M), 2)
        y = torch.empty_like(R)
        t_app = _ms(lambda: api.ilu0_apply(ctx, mesh, M, R, y=y), 5)
        st = api.GmresState(ctx, mesh, restart)
        _, info = api.gmres_solve(ctx, mesh, K, M, R, restart, rtol, state=st)
        t_gm = _ms(lambda: api.gmres_solve(ctx, mesh, K, M, R, restart, rtol, state=st))
        out[name] = {"levels": mesh.n_levels, "factor_ms": t_fac, "apply_ms": t_app, "gmres_iters": info["iters"],
                     "gmres_ms": t_gm}
        if name == "mdf":
            out[name]["ordering_s"] = t_mdf
        st.close()
        del K, M, R, y
        torch.cuda.empty_cache()
    return out


def extra_ras(ctx, hmesh, spec, mats, F, G, restart, rtol=1e-10, subs=(1, 2, 4, 8), deltas=(0, 1)):
    """The paper's restricted additive Schwarz preconditioner with N slab
    subdomains on one GPU (FP64): GMRES iterations against N and delta."""
    import torch
    from paper_1605_01020_amd import api, F64
    A, B, C, D = mats
    fac = api.condense(ctx, A, B, C, D, F, prec=F64)
    mesh = api.Mesh(ctx, hmesh.elem_faces(), hmesh.n_face, spec.b)
    K, R = api.assemble(ctx, mesh, Ke=fac["Ke"], r=fac["r"], G=G, prec=F64)
    del fac
    out = {}
    st = api.GmresState(ctx, mesh, restart)
    for n_sub in subs:
        for delta in deltas:
            ras = api.Ras(ctx, mesh, hmesh.face_slabs(n_sub), delta)
            Ml = ras.factor(K, prec=F64)
            t_fac = _ms(lambda: ras.factor(K, prec=F64, Mloc=Ml))
            y = torch.empty_like(R)
            t_app = _ms(lambda: ras.apply(Ml, R, y=y), 5)
            st.set_ras(ras)
            _, info = api.gmres_solve(ctx, mesh, K, Ml, R, restart, rtol, state=st, raise_on_fail=False)
            out[f"N{n_sub}_delta{delta}"] = {"gmres_iters": info["iters"], "converged": info["converged"],
                                             "local_rows": ras.n_local_rows, "levels": ras.n_levels,
                                             "factor_ms": t_fac, "apply_ms": t_app}
            st.set_ras(None)
            ras.close()
            del Ml, y
            torch.cuda.empty_cache()
    st.close()
    return out


def device_ceilings(ctx):
    """Measured ceilings (outside any timed region): MFMA loops of the
    instructions the condensation issues, and a STREAM triad over 3 x 2 GiB."""
    import torch
    from paper_1605_01020_amd import api, F64, F32, BF16
    out = {}
    for name, prec in (("mfma_f64_tflops", F64), ("mfma_f32_tflops", F32), ("mfma_bf16_16x16x16_tflops", BF16)):
        out[name], sink = api.probe_mfma(ctx, prec)
        del sink
    out["triad_gbps"], arrays = api.probe_triad(ctx)
    del arrays
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--forms", default="mixed,bf16,fp64",
                    help="mixed: FP32 condensation; bf16: BF16-operand condensation; fp64: plain FP64")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the FP64-1e-10, RHS-only, ordering, RAS and batched measurements")
    ap.add_argument("--dims", default="16,16,8")
    ap.add_argument("--p", type=int, default=3)
    ap.add_argument("--workload", default="subdomain", choices=["subdomain", "batch", "serving"])
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--requests", type=int, default=2000, help="serving: measured requests per load")
    ap.add_argument("--serve-warmup", type=int, default=200, help="serving: warm-up requests per load")
    ap.add_argument("--loads", default="0.5,0.7,0.9", help="serving: arrival rates as fractions of capacity")
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--capacity-requests", type=int, default=500,
                    help="serving: closed-loop requests that measure capacity")
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="first run a plain device copy of this many GiB (reference for HBM counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the solve is one subdomain on one MI355X; "
              "multi-GPU runs (RAS across subdomains) are not part of this build.", file=sys.stderr)
        sys.exit(2)

    if args.copy_probe_gib > 0:
        import torch
        nbytes = int(args.copy_probe_gib * 2 ** 30)
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        _log(f"copy probe: 3 copies of {nbytes} bytes")
        del src, dst
        torch.cuda.empty_cache()
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serving":
        return bench_serving(args)

    import numpy as np
    import torch
    from paper_1605_01020_amd import api, F64, F32, BF16
    from paper_1605_01020_amd.solver import NewtonStepSolver, StepTimer
    import synth.device as sd
    from synth import StructuredHexMesh, ElementSpec
    from synth.matrices import workload

    wl = workload(1)
    dims = tuple(int(v) for v in args.dims.split(","))
    spec = ElementSpec(args.p)
    hmesh = StructuredHexMesh(*dims)
    E, n, t = hmesh.n_elem, spec.n, spec.t
    torch.cuda.set_device(0)
    ctx = api.Context(0)
    from paper_1605_01020_amd.autotune import apply_tuning
    apply_tuning(ctx)
    mesh = api.Mesh(ctx, hmesh.elem_faces(), hmesh.n_face, spec.b)
    print(f"[bench] {dims} p={args.p}: E={E} n={n} t={t} faces={hmesh.n_face} nnzb={mesh.nnzb}", file=sys.stderr,
          flush=True)
    mats_d = sd.gen_blocks(spec, wl.seed, 0, E, which="ABCD")
    n_rhs = wl.n_rhs
    Fs = [sd.gen_blocks(spec, wl.seed, 0, E, which="F", rhs=k)["F"] for k in range(n_rhs)]
    Gs = [sd.gen_trace_rhs(spec, wl.seed, 0, hmesh.n_face, rhs=k) for k in range(n_rhs)]
    torch.cuda.synchronize()
    print("[bench] inputs generated in HBM", file=sys.stderr, flush=True)
    A, B, C, D = mats_d["A"], mats_d["B"], mats_d["C"], mats_d["D"]

    results = {}
    for form in [f for f in args.forms.split(",") if f]:
        solver = NewtonStepSolver(ctx, mesh, n, restart=wl.restart)
        lat, cond_ms, iters, rho, steps_ref = [], [], [], [], []

        def step(k, record):
            timer = StepTimer(True)
            F, G = Fs[k % n_rhs], Gs[k % n_rhs]
            if form == "fp64":
                z, u, info = solver.solve_fp64(A, B, C, D, F, G, rtol=args.tol, timer=timer)
            else:
                z, u, info = solver.solve_mixed(A, B, C, D, F, G, tol=args.tol, prec=BF16 if form == "bf16" else F32,
                                                timer=timer)
            if record:
                cond_ms.append(info["phases_ms"].get("condense", float("nan")))
                iters.append(info["iters"])
                steps_ref.append(info.get("refine_steps", 0))
            return z, u, info

        for k in range(args.warmup):
            step(k, False)
        torch.cuda.synchronize()
        print(f"[bench] {form}: warmup done", file=sys.stderr, flush=True)
        t_start = time.perf_counter()
        for k in range(args.steps):
            t0 = time.perf_counter()
            z, u, info = step(args.warmup + k, True)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - t0) * 1e3)
        torch.cuda.synchronize()
        total = time.perf_counter() - t_start
        ctx.sync_status()
        # accuracy of the last step, outside the timed region
        k_last = (args.warmup + args.steps - 1) % n_rhs
        _, _, sums = api.residual_full(ctx, mesh, A, B, C, D, Fs[k_last], Gs[k_last], z, u)
        s = sums.cpu().numpy()
        rho_full = math.sqrt((s[0] + s[1]) / (s[2] + s[3]))
        ms = total * 1e3 / args.steps
        cms = float(np.mean(cond_ms))
        results[form] = {"solves_per_s": 1e3 / ms, "ms_per_step": ms,
                         "elements_condensed_per_s": E / (cms * 1e-3), "condense_ms": cms,
                         "gmres_iters": iters, "refine_steps": steps_ref, "rho_full": rho_full,
                         "lat_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
                         "phases_ms_last": info["phases_ms"]}
        print(f"[bench] {form}: {ms:.1f} ms/step, condense {cms:.1f} ms, iters {iters}, rho_full {rho_full:.2e}",
              file=sys.stderr, flush=True)
        del solver
        torch.cuda.empty_cache()

    _log("device ceilings: MFMA loops and STREAM triad")
    ceilings = device_ceilings(ctx)
    _log(f"  {ceilings}")

    extras = {}
    if not args.no_extras:
        mats = (A, B, C, D)
        _log("extra: fp64 form at 1e-10")
        extras["fp64_rtol_1e-10"] = extra_fp64_tight(ctx, mesh, n, mats, Fs, Gs, wl.restart)
        _log("extra: rhs-only solves with retained factors")
        extras["rhs_solves"] = extra_rhs_solves(ctx, mesh, n, mats, Fs, Gs, wl.restart)
        _log("extra: minimal-residual Newton initial guess")
        extras["mr_guess"] = extra_mr_guess(ctx, mesh, n, mats, Fs[0], Gs[0], wl.restart)
        _log("extra: IEDG trace numbering")
        extras["iedg_trace"] = extra_iedg(ctx, hmesh, spec, mats, Fs[0], wl.restart, wl.seed)
        _log("extra: orderings (natural, colour, mdf)")
        extras["orderings_fp64_rtol_1e-10"] = extra_orderings(ctx, hmesh, spec, mats, Fs[0], Gs[0], wl.restart)
        _log("extra: restricted additive Schwarz")
        extras["ras_fp64_rtol_1e-10"] = extra_ras(ctx, hmesh, spec, mats, Fs[0], Gs[0], wl.restart)
        del A, B, C, D, mats, mats_d, Fs, Gs
        torch.cuda.empty_cache()
        from paper_1605_01020_amd import F64 as _F64
        _log("extra: batched form, FP32-mixed and FP64")
        bf = {"f32": batch_form(ctx, F32, args), "f64": batch_form(ctx, _F64, args)}
        bf["speedup_mixed_vs_fp64"] = bf["f32"]["solves_per_s"] / bf["f64"]["solves_per_s"]
        extras["batch_24_meshes"] = bf
        _log("extra: serving form (reduced: 0.7 x capacity, 40 warm-up + 120 measured requests)")
        extras["serving_reduced"] = serving_sweep(ctx, [0.7], 40, 120, args.slots, args.budget_gb, n_cap=80)

    head = "mixed" if "mixed" in results else "fp64"
    r = results[head]
    flops = condense_flops(n, t) * E
    peak = FP32_PEAK_TFLOPS if head == "mixed" else FP64_PEAK_TFLOPS
    achieved = flops / (r["condense_ms"] * 1e-3) / 1e12
    measured_peak = ceilings["mfma_f32_tflops" if head == "mixed" else "mfma_f64_tflops"]
    traffic = None
    if head == "mixed" and dims == (16, 16, 8) and args.p == 3:
        traffic = measured_traffic(CONDENSE_SOURCES, "hbm_traffic_16x16x8_p3.md")
    out = {
        "metric": "Newton-step solves/s at relative residual 1e-8 (mixed FP32/FP64 form; FP64 form beside it)",
        "value": r["solves_per_s"],
        "unit": "Newton-step solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head == "mixed" else "f64",
        "data": "synthetic (seeded Philox element blocks generated in HBM)",
        "config": {"workload": f"IEDG Newton-step trace solve, {dims[0]}x{dims[1]}x{dims[2]} hex mesh, p={args.p}, "
                               f"E={E}, n={n}, t={t}, N_t={hmesh.n_face * spec.b}, GMRES(100)+BILU(0), 10 RHS",
                   "form": head, "tol": args.tol},
        "elements_condensed_per_s": r["elements_condensed_per_s"],
        "lat_ms": r["lat_ms"],
        "forms": results,
        "roofline": {"bound": "mfma", "kernel": "condense", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "flops_per_launch": flops,
                     "measured_peak": measured_peak, "frac_of_measured": achieved / measured_peak},
        "device_ceilings": ceilings,
    }
    out.update(extras)
    if "fp64" in results and "mixed" in results:
        out["speedup_mixed_vs_fp64"] = results["mixed"]["solves_per_s"] / results["fp64"]["solves_per_s"]
    if "fp64" in results and "bf16" in results:
        out["speedup_bf16_vs_fp64"] = results["bf16"]["solves_per_s"] / results["fp64"]["solves_per_s"]
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl.seed, wl.restart)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
