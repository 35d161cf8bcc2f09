"""Bitwise reproducibility of every output of the regression path.

FP32 data with s <= 1024 and r1 <= 1024 takes the bucket-owner sketch, whose
sums are formed in an order fixed by the random streams; with
FCT_FLAG_DETERMINISTIC larger r1 is split over workgroups the same way.  The
other steps are deterministic by construction (one thread or a fixed tree per
value).  Two runs, each in a fresh context on freshly uploaded inputs, must
give the same bits for Y, R, lambda, sum lambda, the kept rows and their
weights, and x.
"""
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


def run_once(F, A, b, w, flags):
    ctx = F.Context(0)
    try:
        Ad, bd = torch.from_numpy(A).cuda(), torch.from_numpy(b).cuda()
        Y, R = F.fct_sketch(ctx, Ad, bd, w.s, w.r1, w.seed, flags=flags)
        lam, p, tot = F.l1_sample_probs(ctx, Ad, bd, R, w.r2, w.seed, w.s_out)
        cap = 2 * w.s_out + 8 * int(np.sqrt(w.s_out)) + 1024
        idx, wt, S = F.l1_select(ctx, lam, tot, w.s_out, w.seed, cap)
        prm = F.params(s=w.s, r1=w.r1, r2=w.r2, s_out=w.s_out, seed=w.seed, flags=flags)
        x, obj, S2 = F.l1_regress(ctx, Ad, bd, prm, eps=w.eps)
        torch.cuda.synchronize()
        out = dict(Y=Y.cpu().numpy(), R=R.cpu().numpy(), lam=lam.cpu().numpy(), p=p.cpu().numpy(),
                   tot=tot.cpu().numpy(), idx=idx.cpu().numpy()[:S], wt=wt.cpu().numpy()[:S],
                   x=np.asarray(x), obj=np.array([obj]), S=np.array([S, S2]))
    finally:
        ctx.close()
    return out


@pytest.mark.parametrize("n,r1,flags", [(1 << 21, 1024, 0), (1 << 20, 2048, "det")])
def test_two_runs_same_bits(F, n, r1, flags):
    w = synth.scaled(synth.LARGE, n, r1=r1)
    fl = F.FCT_FLAG_DETERMINISTIC if flags == "det" else 0
    A, b, _ = synth.generate(w)
    print(f"determinism n={n} r1={r1} flags={fl}", flush=True)
    a1 = run_once(F, A, b, w, fl)
    a2 = run_once(F, A, b, w, fl)
    for k in a1:
        v1, v2 = a1[k], a2[k]
        assert v1.shape == v2.shape, k
        assert v1.tobytes() == v2.tobytes(), k
