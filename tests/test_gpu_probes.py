"""The measured-ceiling probes behind the roofline report (iedg_probe_*):
the MFMA loop runs every iteration (each thread's accumulator sum is exact:
operands of one), and the STREAM triad writes b + s c exactly (s = 2: the
product is exact) on a length that leaves a ragged last workgroup."""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu
api = pytest.importorskip("paper_1605_01020_amd.api")


def _say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = api.Context()
    yield c
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec,k", [(0, 4), (1, 4), (2, 16)])
def test_mfma_probe_runs_every_iteration(ctx, prec, k):
    _say(f"mfma probe prec={prec}")
    iters = 100
    tf, sink = api.probe_mfma(ctx, prec, n_wg=6, iters=iters, reps=2)
    assert tf > 0
    # 8 chains of 4 accumulator entries a lane, each K iters
    assert torch.all(sink == 32.0 * k * iters).item()


def test_triad_probe_exact_and_ragged(ctx):
    n = 2 * (1024 * 37 + 5)
    _say(f"triad probe n={n}")
    g = torch.Generator(device="cuda").manual_seed(5)
    b = torch.randn(n, generator=g, device="cuda", dtype=torch.float64)
    c = torch.randn(n, generator=g, device="cuda", dtype=torch.float64)
    a = torch.full_like(b, np.nan)
    gbps, _ = api.probe_triad(ctx, n=n, s=2.0, reps=2, arrays=(a, b, c))
    assert gbps > 0
    assert torch.equal(a, b + 2.0 * c)


def test_probes_reject_bad_arguments(ctx):
    x = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(api.IedgError):
        api.probe_triad(ctx, n=7, arrays=(x, x, x), reps=1)
    with pytest.raises(api.IedgError):
        api.probe_mfma(ctx, 0, n_wg=1, iters=0, reps=1)
    with pytest.raises(api.IedgError):
        api.probe_mfma(ctx, 7, n_wg=1, iters=1, reps=1)
