"""The batched form (many instances of uneven n and d in one captured graph).

Each instance of a batch drawn like the batching workload (n in [2^14, 2^20],
d in {8, 16, 32, 64}, r1 = 8 d ceil(log2 d), s_out = 250 q) must give what
the single-instance path gives with the same parameters: the same coreset
size and an objective equal to solver precision (the batched solve runs on
one workgroup per instance, the single path on several, so their sums are
rounded in different orders).  Solver precision: the smoothed objective
with eta at its floor, 1e-6 of the mean weighted residual, exceeds the exact
one by at most 1e-6 of the objective, so each solve ends within that of the
coreset optimum.  A replay of the
captured graph must reproduce the first call, autotuned block sizes must be
among the candidates, and a small instance must meet the (1 + eps) bound
against the exact LP optimum.
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import l1

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    from conftest import ensure_built
    ensure_built()
    from paper_1207_4684_amd import fctl1
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return fctl1


@pytest.fixture(scope="module")
def ctx(F):
    c = F.Context(0)
    yield c
    c.close()


def make_batch(F, count, autotune_every=2):
    items, hosts = [], []
    for i, w in enumerate(synth.batch_instances(count)):
        A, b, _ = synth.generate(w)
        s = 0 if i % autotune_every == 0 else w.s
        prm = F.params(s=s, r1=w.r1, r2=w.r2, s_out=w.s_out, seed=w.seed)
        items.append(dict(A=torch.from_numpy(A).cuda(), b=torch.from_numpy(b).cuda(), prm=prm, w=w))
        hosts.append((A, b))
    return items, hosts


def test_batched_matches_single_instances_and_replays(F, ctx):
    items, _ = make_batch(F, 16)
    res, st = F.l1_regress_batched(ctx, items, eps=0.05)
    assert st == 0, [r["status"] for r in res]
    res2, st2 = F.l1_regress_batched(ctx, items, eps=0.05)   # graph replay
    assert st2 == 0
    for it, r, r2 in zip(items, res, res2):
        w = it["w"]
        assert r["s"] in (64, 128, 256, 512)
        prm = F.params(s=r["s"], r1=w.r1, r2=w.r2, s_out=w.s_out, seed=w.seed)
        x1, _, S1 = F.l1_regress(ctx, it["A"], it["b"], prm, eps=0.05)
        f1 = F.fct_l1_objective(ctx, it["A"], it["b"], x1)
        fb = F.fct_l1_objective(ctx, it["A"], it["b"], r["x"])
        fb2 = F.fct_l1_objective(ctx, it["A"], it["b"], r2["x"])
        print(f"n={w.n} d={w.d} s={r['s']} S={r['S']} batched/single {fb / f1 - 1:.2e}")
        assert r["S"] == S1 and r2["S"] == S1
        assert abs(fb / f1 - 1) <= 1e-6 and abs(fb2 / fb - 1) <= 1e-6


def test_batched_one_plus_eps_small_instance(F, ctx):
    w = synth.scaled(synth.batch_instances(1)[0], 16384, d=8, r1=8 * 8 * 3, s_out=250 * 9)
    A, b, _ = synth.generate(w)
    prm = F.params(s=0, r1=w.r1, r2=w.r2, s_out=w.s_out, seed=w.seed)
    it = dict(A=torch.from_numpy(A).cuda(), b=torch.from_numpy(b).cuda(), prm=prm)
    res, st = F.l1_regress_batched(ctx, [it, it], eps=0.05)
    assert st == 0
    At, b64 = A.T.astype(np.float64), b.astype(np.float64)
    _, fopt = l1.lp(At, b64)
    for r in res:
        assert l1.objective(At, b64, np.array(r["x"])) <= (1 + 0.05) * fopt


def test_solver_shapes_agree_on_ill_conditioned_coreset(F, ctx, monkeypatch):
    """Instance 206 of the batching workload (n = 25110, d = 32): its coreset
    makes the reweighted systems badly conditioned near the optimum.  One
    workgroup streaming every row (the batched shape) and the cooperative grid
    must both end within the smoothing bound of the exact LP optimum."""
    import math
    w = synth.batch_instances(207)[206]
    A, b, _ = synth.generate(w)
    prm = F.params(s=256, r1=w.r1, r2=w.r2, s_out=w.s_out, seed=w.seed)
    cap = min(w.n, 2 * w.s_out + 8 * int(math.sqrt(w.s_out)) + 1024)
    At, bt, wt, idx, S = F.l1_coreset(ctx, torch.from_numpy(A).cuda(), torch.from_numpy(b).cuda(),
                                      prm, cap)
    Ah = At.double().cpu().numpy()
    bh = bt.double().cpu().numpy()
    wh = wt.cpu().numpy()
    _, fopt = l1.lp(Ah, bh, wh)
    x_many, o_many = F.l1_solve(ctx, At.t(), bt, wt)
    monkeypatch.setenv("FCTL1_IRLS_WGS", "1")
    x_one, o_one = F.l1_solve(ctx, At.t(), bt, wt)
    for x in (x_many, x_one):
        f = l1.objective(Ah, bh, x, wh)
        print(f"S={S} f/fopt - 1 = {f / fopt - 1:.3e}")
        assert f <= fopt * (1 + 1e-6)
