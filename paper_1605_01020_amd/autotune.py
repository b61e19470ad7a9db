"""Measured choice of the condensation kernel's sub-panel and panel widths.

The panel factorisation of the condensation kernel keeps sub-panels of 8
or 16 columns in registers, and its Crout updates work on panels of 64 or
(FP32 storage only) 128 columns, which set the GEMM tile shapes.  For each
precision and element size the tuner times every combination on a
device-generated sample of elements and keeps the fastest; the table is
stored as tuning.json beside this file and applied with iedg_set_leaf_width
and iedg_set_panel_width.

    python -m paper_1605_01020_amd.autotune          # measure and write
"""
import json
import os
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
TUNING_PATH = os.path.join(_HERE, "tuning.json")
LEAF_CHOICES = (8, 16)
PANEL_CHOICES = {"f32": (64, 128), "bf16": (64, 128), "f64": (64,)}
PREC_NAME = {0: "f64", 1: "f32", 2: "bf16"}


def _time_condense(ctx, spec, d, prec, reps):
    import torch
    from . import api
    out = api.condense(ctx, d["A"], d["B"], d["C"], d["D"], d["F"], prec=prec)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        api.condense(ctx, d["A"], d["B"], d["C"], d["D"], d["F"], prec=prec, out=out)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ctx.sync_status()
    return min(ts)


def tune(ctx, ps=(2, 3, 4), precs=None, n_elem=512, reps=3, seed=1605010203, log=print):
    import torch
    from . import api
    from ._lib import F32, F64, BF16
    from synth import ElementSpec
    import synth.device as sd
    precs = (F32, F64, BF16) if precs is None else precs
    table = {"n_elem": n_elem, "entries": []}
    for p in ps:
        spec = ElementSpec(p)
        d = sd.gen_blocks(spec, seed, 0, n_elem, which="ABCDF")
        for prec in precs:
            best = None
            times = {}
            pn = PREC_NAME[int(prec)]
            for ct in PANEL_CHOICES[pn]:
                api.set_panel_width(ctx, spec.n, ct, prec=prec)
                for lw in LEAF_CHOICES:
                    api.set_leaf_width(ctx, spec.n, lw, prec=prec)
                    ms = _time_condense(ctx, spec, d, prec, reps)
                    times[(lw, ct)] = ms
                    log(f"p={p} n={spec.n} prec={pn} sub-panel {lw} panel {ct}: {ms:.2f} ms for {n_elem} elements")
                    if best is None or ms < times[best]:
                        best = (lw, ct)
            api.set_leaf_width(ctx, spec.n, best[0], prec=prec)
            api.set_panel_width(ctx, spec.n, best[1], prec=prec)
            table["entries"].append({"p": p, "n": spec.n, "prec": pn, "leaf_width": best[0], "panel_width": best[1],
                                     "ms": {f"{k[0]}/{k[1]}": v for k, v in times.items()}})
        del d
        torch.cuda.empty_cache()
    return table


def apply_tuning(ctx, path=TUNING_PATH):
    """Apply a stored table (no-op when none has been measured)."""
    from . import api
    if not os.path.exists(path):
        return None
    with open(path) as f:
        table = json.load(f)
    from ._lib import F32, F64, BF16
    for e in table.get("entries", []):
        prec = {"f64": F64, "bf16": BF16}.get(e.get("prec"), F32)
        api.set_leaf_width(ctx, int(e["n"]), int(e["leaf_width"]), prec=prec)
        if "panel_width" in e:
            api.set_panel_width(ctx, int(e["n"]), int(e["panel_width"]), prec=prec)
    return table


def main():
    import torch
    from . import api
    torch.cuda.set_device(0)
    ctx = api.Context(0)
    table = tune(ctx, log=lambda m: print(f"[autotune] {m}", flush=True))
    out = sys.argv[1] if len(sys.argv) > 1 else TUNING_PATH
    with open(out, "w") as f:
        json.dump(table, f, indent=1)
    print(f"[autotune] wrote {out}", flush=True)


if __name__ == "__main__":
    main()
