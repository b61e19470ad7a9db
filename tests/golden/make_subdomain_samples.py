"""Write sampled FP64 oracle values of the full-size subdomain solve.

Workload: 16x16x8 structured hex mesh, p = 3 (2,048 elements, n = 1,280,
t = 480, 6,656 faces of b = 80 trace dofs, N_t = 532,480), seed 1605010201,
right-hand side 0.  The oracle (oracle/, plain FP64) is run streamed, element
by element, so its inputs never need to be resident at once:

  pass 1: generate each element's blocks (synth), condense it
          (oracle.condense_element: K_e, r_e), drop the blocks;
  trace:  oracle.assemble, oracle.bilu0 (colour order), oracle.gmres with
          restart 100 to a true relative residual of 1e-12;
  pass 2: regenerate A_e, B_e, F_e and recover z_e (oracle.backsolve_element).

Stored (tests/golden/subdomain_16x16x8_p3_rhs0.json): ||uhat||, ||z||, 512
seeded entries of uhat, the full z of three elements, the GMRES iteration
count and the true relative residual.  Only oracle/ and synth/ are called.
Takes about an hour on 8 cores and ~12 GB of host memory.

    python tests/golden/make_subdomain_samples.py [--procs 4]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

DIMS, P, CONFIG, RHS = (16, 16, 8), 3, 1, 0
SAMPLE_ELEMS = (0, 1037, 2047)
N_UHAT_SAMPLES = 512
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "subdomain_16x16x8_p3_rhs0.json")


def _limit_blas(threads):
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(threads)
    except Exception:
        pass


def _condense_range(args):
    e0, e1, seed, threads = args
    _limit_blas(threads)
    import oracle
    from synth import ElementSpec, element_inputs
    spec = ElementSpec(P)
    Ks, rs = [], []
    for e in range(e0, e1):
        blk = element_inputs(spec, seed, 0, e, rhs=RHS)
        Ke, re, _ = oracle.condense_element(blk["A"], blk["B"], blk["C"], blk["D"], blk["F"])
        Ks.append(Ke)
        rs.append(re)
    return e0, Ks, rs


def _backsolve_range(args):
    e0, e1, seed, threads, uhat_parts = args
    _limit_blas(threads)
    import oracle
    from synth import ElementSpec, element_inputs
    spec = ElementSpec(P)
    zs = []
    for k, e in enumerate(range(e0, e1)):
        blk = element_inputs(spec, seed, 0, e, rhs=RHS, which="ABF")
        zs.append(oracle.backsolve_element(blk["A"], blk["B"], blk["F"], uhat_parts[k]))
    return e0, zs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=4)
    ap.add_argument("--chunk", type=int, default=16)
    args = ap.parse_args()
    import multiprocessing as mp
    import oracle
    from oracle.assembly import matvec
    from synth import StructuredHexMesh, ElementSpec, trace_rhs
    from synth.matrices import workload
    seed = workload(CONFIG).seed
    mesh = StructuredHexMesh(*DIMS)
    spec = ElementSpec(P)
    tm = oracle.TraceMesh(mesh.elem_faces(), mesh.n_face, spec.b)
    E = mesh.n_elem
    threads = max(1, (os.cpu_count() or 8) // args.procs)
    jobs = [(e0, min(E, e0 + args.chunk), seed, threads) for e0 in range(0, E, args.chunk)]
    t0 = time.time()
    Ks, rs = [None] * E, [None] * E
    with mp.get_context("fork").Pool(args.procs) as pool:
        for done, (e0, k_part, r_part) in enumerate(pool.imap_unordered(_condense_range, jobs)):
            Ks[e0:e0 + len(k_part)] = k_part
            rs[e0:e0 + len(r_part)] = r_part
            print(f"condensed chunk {done + 1}/{len(jobs)} ({time.time() - t0:.0f} s)", flush=True)
    G = trace_rhs(spec, seed, 0, mesh.n_face, rhs=RHS)
    K, R = oracle.assemble(tm, Ks, rs, G)
    del Ks, rs
    order = oracle.greedy_colour_order(tm)
    fac = oracle.bilu0(tm, K, order)
    print(f"bilu0 done ({time.time() - t0:.0f} s)", flush=True)
    uhat, info = oracle.gmres(lambda v: matvec(tm, K, v), lambda v: oracle.bilu0_apply(tm, fac, v), R,
                              restart=100, rtol=1e-12)
    print(f"gmres: {info['iters']} iterations, rel resid {info['rel_resid']:.3e} ({time.time() - t0:.0f} s)",
          flush=True)
    del K, fac
    jobs2 = [(e0, e1, seed, threads, [uhat[tm.element_dofs(e)] for e in range(e0, e1)]) for e0, e1, _, _ in jobs]
    z = [None] * E
    with mp.get_context("fork").Pool(args.procs) as pool:
        for done, (e0, zp) in enumerate(pool.imap_unordered(_backsolve_range, jobs2)):
            z[e0:e0 + len(zp)] = zp
            if (done + 1) % 16 == 0:
                print(f"back-substituted chunk {done + 1}/{len(jobs2)} ({time.time() - t0:.0f} s)", flush=True)
    zn = float(np.sqrt(sum(float(v @ v) for v in z)))
    rng = np.random.default_rng(16050102)
    idx = np.sort(rng.choice(tm.n_trace, N_UHAT_SAMPLES, replace=False))
    out = {
        "what": "FP64 oracle solve of the 16x16x8 p=3 subdomain, right-hand side 0 (streamed; see the script)",
        "dims": list(DIMS), "p": P, "seed": seed, "rhs": RHS, "ordering": "colour", "restart": 100,
        "rtol": 1e-12, "gmres_iters": int(info["iters"]), "rel_resid": float(info["rel_resid"]),
        "uhat_norm": float(np.linalg.norm(uhat)), "z_norm": zn,
        "uhat_index": [int(i) for i in idx], "uhat_value": [float(uhat[i]) for i in idx],
        "z_elements": {str(e): [float(v) for v in z[e]] for e in SAMPLE_ELEMS},
        "seconds": time.time() - t0,
    }
    with open(OUT, "w") as f:
        json.dump(out, f)
    print(f"wrote {OUT} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
