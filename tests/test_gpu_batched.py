"""The batched form (many instances of uneven n and d in one captured graph)
against the oracle.

A batch drawn like the batching workload (n in [2^14, 2^20], d in
{8, 16, 32, 64}, r1 = 8 d ceil(log2 d), s_out = 250 q; every other instance
leaves s to the library) runs once with every instance's R, lambda and kept
rows copied out.  For each instance the oracle then checks, at the s the
batch used: R against the Gram matrix of the oracle's sketch, lambda over all
rows from the batch's R, the kept rows exactly from the batch's lambda, and
the (1 + eps) objective (the oracle's FP64 sum) against the oracle's LP
optimum or weak-duality bound.  A replay of the captured graph must keep the
same coresets, and the library's block size must follow its documented rule.
The batched solve gives the costliest instances several workgroups each (a
barrier per instance) and the others one; every instance must agree with the
single-instance path (cooperative grid) on the same parameters.
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import basis, fct, l1, philox, sampling

pytestmark = pytest.mark.gpu

BATCH = 8


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


def capacity(w):
    return min(w.n, 2 * w.s_out + 8 * int(math.sqrt(w.s_out)) + 1024)


def make_batch(F, count, library_s_every=2, outputs=False):
    items, hosts = [], []
    for i, w in enumerate(synth.batch_instances(count)):
        A, b, _ = synth.generate(w)
        s = 0 if i % library_s_every == 0 else w.s
        prm = F.params(s=s, r1=w.r1, r2=w.r2, s_out=w.s_out, seed=w.seed)
        it = dict(A=torch.from_numpy(A).cuda(), b=torch.from_numpy(b).cuda(), prm=prm, w=w)
        if outputs:
            q = w.d + 1
            it["R_out"] = torch.zeros((q, q), dtype=torch.float64, device="cuda")
            it["lambda_out"] = torch.zeros(w.n, dtype=torch.float32, device="cuda")
            it["idx_out"] = torch.full((capacity(w),), -1, dtype=torch.int64, device="cuda")
        items.append(it)
        hosts.append((A, b))
    return items, hosts


def block_size_rule(d):
    t = math.ceil(2 * d * math.log(d))
    s = 64
    while s < t and s < 1024:
        s *= 2
    return s


@pytest.fixture(scope="module")
def batch(F, ctx):
    items, hosts = make_batch(F, BATCH, outputs=True)
    res, st = F.l1_regress_batched(ctx, items, eps=0.05)
    assert st == 0, [r["status"] for r in res]
    torch.cuda.synchronize()
    outs = [dict(R=it["R_out"].cpu().numpy().T.copy(), lam=it["lambda_out"].cpu().numpy(),
                 idx=it["idx_out"].cpu().numpy()) for it in items]
    res2, st2 = F.l1_regress_batched(ctx, items, eps=0.05)   # graph replay
    assert st2 == 0
    return items, hosts, res, res2, outs


def test_batched_replay_and_block_size(F, ctx, batch):
    items, _, res, res2, _ = batch
    for it, r, r2 in zip(items, res, res2):
        w = it["w"]
        expect = block_size_rule(w.d) if it["prm"].s == 0 else w.s
        assert r["s"] == expect and r2["s"] == expect
        assert r2["S"] == r["S"]
        assert abs(r2["obj"] / r["obj"] - 1) <= 1e-6


def test_batched_matches_single_instance_path(F, ctx, batch):
    items, _, res, _, _ = batch
    for it, r in zip(items, res):
        w = it["w"]
        prm = F.params(s=r["s"], r1=w.r1, r2=w.r2, s_out=w.s_out, seed=w.seed)
        x, obj, S = F.l1_regress(ctx, it["A"], it["b"], prm, eps=0.05)
        # sketches with r1 > 1024 add in LDS atomically, so a row at its
        # threshold may fall either way: then the coresets differ by a row
        assert abs(S - r["S"]) <= 2
        tol = 1e-6 if S == r["S"] else 1e-3
        assert abs(r["obj"] / obj - 1) <= tol, (w.n, w.d, r["obj"] / obj - 1)


@pytest.mark.parametrize("i", range(BATCH))
def test_batched_instance_against_oracle(F, ctx, batch, i):
    items, hosts, res, _, outs = batch
    w, r, o = items[i]["w"], res[i], outs[i]
    A, b = hosts[i]
    X = np.hstack([A.T.astype(np.float64), -b.astype(np.float64)[:, None]])
    print(f"instance {i}: n={w.n} d={w.d} s={r['s']} S={r['S']}", flush=True)
    # R: R^T R against the oracle sketch's Gram matrix, with the sketch gate's
    # bound carried through (the batch's FP64 sketch is within 1e-5 S_i of Yo)
    Yo, S = fct.pi1_apply(X, r["s"], w.r1, w.seed, return_scale=True)
    R = o["R"]
    assert np.all(np.diag(R) > 0) and np.allclose(np.tril(R, -1), 0)
    G = Yo.T @ Yo
    aY = (S[:, None] * np.abs(Yo)).sum(axis=0)
    bound = 1e-5 * (aY[:, None] + aY[None, :]) + 1e-10 * float(S @ S) + 1e-12 * np.abs(G).max()
    assert np.all(np.abs(R.T @ R - G) <= bound), float(np.max(np.abs(R.T @ R - G) / bound))
    # lambda over all rows, from the batch's R
    M = basis.m_matrix(R, w.seed, w.r2)
    ref = sampling.row_norm_estimates(X, M)
    scale = (np.abs(X) @ np.abs(M)).max(axis=1)
    assert np.all(np.abs(o["lam"] - ref) <= 1e-5 * scale)
    # the kept rows, from the batch's lambda (FP64 decisions on both sides)
    lam = o["lam"].astype(np.float64)
    p = sampling.probabilities(lam, w.s_out, lam.sum())
    keep = philox.sample_words(w.seed, w.n) < sampling.thresholds(p)
    oidx = np.flatnonzero(keep)
    assert r["S"] == oidx.size
    assert np.array_equal(o["idx"][:oidx.size], oidx)
    # (1 + eps): f(x) by the oracle against the optimum or a certified bound
    At, b64 = A.T, b.astype(np.float64)
    f = l1.objective(At, b64, np.array(r["x"]), chunk=1 << 18)
    if w.n <= 20000:
        lower = l1.lp(At.astype(np.float64), b64)[1]
    else:
        x0, _ = F.l1_solve(ctx, items[i]["A"], items[i]["b"],
                           torch.ones(w.n, dtype=torch.float64, device="cuda"), iters=120)
        lower = l1.dual_lower_bound(At, b64, x0, threads=16, stop_at=f / 1.025)
    print(f"instance {i}: f / lower = {f / lower:.6f}")
    assert f <= 1.05 * lower, f / lower


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


def test_solver_shapes_agree_on_ill_conditioned_coreset(F, ctx):
    """Instance 206 of the batching workload (n = 25110, d = 32): its coreset
    makes the reweighted systems badly conditioned near the optimum.  One
    workgroup streaming every row (the batched shape) and the cooperative grid
    must both end within the smoothing bound of the exact LP optimum."""
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
    one = F.Context(0)
    try:
        one.set_option(F.FCT_OPT_SOLVE_WGS, 1)
        x_one, o_one = F.l1_solve(one, At.t(), bt, wt)
    finally:
        one.close()
    for x in (x_many, x_one):
        f = l1.objective(Ah, bh, x, wh)
        print(f"S={S} f/fopt - 1 = {f / fopt - 1:.3e}")
        assert f <= fopt * (1 + 1e-6)
