"""The entry point that allocates nothing (l1_sample_probs_noalloc) against
the existing sampling-pass entry point (l1_sample_probs / _ex) through the C
ABI: bitwise-equal lambda, probabilities and sum on two calls in a row, the
second with a smaller input, for the FP32, BF16 and FP64 streams and both
Pi2 kinds; and the capacity error when the pass-2 grid would outgrow the
static scratch."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    from conftest import ensure_built
    ensure_built()
    from paper_1207_4684_amd import fctl1
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return fctl1


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _same_bits(x, y):
    torch.cuda.synchronize()
    return torch.equal(x.view(torch.int32) if x.dtype == torch.float32 else x.view(torch.int64),
                       y.view(torch.int32) if y.dtype == torch.float32 else y.view(torch.int64))


@pytest.mark.parametrize("kind", ["f32", "bf16", "f64", "gaussian"])
def test_noalloc_matches_sample_probs(F, kind):
    ctx = F.Context(0)
    try:
        for n, d, r2 in ((300000, 16, 16), (70001, 7, 8)):   # second call smaller
            print(f"noalloc {kind} n={n} d={d}", flush=True)
            w = synth.scaled(synth.TALL, n, d=d, seed=d)
            A, b, _ = synth.generate(w)
            if kind == "f64":
                A, b = A.astype(np.float64), b.astype(np.float64)
            Ad, bd = dev(A), dev(b)
            _, R = F.fct_sketch(ctx, Ad, bd, 256, 512, 5)
            if kind == "bf16":
                Ad, bd = F.fct_to_bf16(ctx, Ad), F.fct_to_bf16(ctx, bd)
            flags = F.FCT_FLAG_GAUSSIAN_PI2 if kind == "gaussian" else 0
            lam_r, p_r, tot_r = F.l1_sample_probs(ctx, Ad, bd, R, r2, 5, 4000, flags=flags)
            lam = torch.full((n,), np.nan, dtype=torch.float32, device="cuda")
            p = torch.full((n,), np.nan, dtype=torch.float32, device="cuda")
            tot = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
            F.l1_sample_probs_noalloc(ctx, Ad, bd, R, r2, 5, 4000, lam, tot, p=p, flags=flags)
            assert _same_bits(lam, lam_r) and _same_bits(p, p_r) and _same_bits(tot, tot_r)
    finally:
        ctx.close()


def test_noalloc_rejects_grid_beyond_scratch(F):
    ctx = F.Context(0)
    try:
        n, d = 2_200_000, 64
        A = torch.randn(d, n, device="cuda")
        b = torch.randn(n, device="cuda")
        R = torch.eye(d + 1, dtype=torch.float64, device="cuda")
        lam = torch.empty(n, device="cuda")
        tot = torch.empty(1, dtype=torch.float64, device="cuda")
        ctx.set_option(F.FCT_OPT_PASS2_WGS, 8000)
        with pytest.raises(F.FctError) as e:
            F.l1_sample_probs_noalloc(ctx, A, b, R, 32, 1, 100, lam, tot)
        assert e.value.status == -6
        ctx.set_option(F.FCT_OPT_PASS2_WGS, 0)
        F.l1_sample_probs_noalloc(ctx, A, b, R, 32, 1, 100, lam, tot)
        lam_r, _, tot_r = F.l1_sample_probs(ctx, A, b, R, 32, 1, 100, want_p=False)
        assert _same_bits(lam, lam_r) and _same_bits(tot, tot_r)
    finally:
        ctx.close()
