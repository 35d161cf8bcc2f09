"""Several coresets from one sampling pass, and sampling with replacement
(the regression figure's caption; the large-scale evaluation's many
solutions in one pass), against the oracle.

* l1_select_draw, Bernoulli, draw k: kept rows and weights bit-exact given
  the GPU's lambda and sum (instance k of stream 3).
* l1_select_draw with replacement, draw k, on synthetic lambda with zeros,
  ragged and large n: every sample's row equals the oracle's inversion of the
  running sums, except where the target lies within rounding of an interval
  end (the two sides add lambda in different orders); weights within 1e-12.
* l1_regress_multi, both kinds: the Bernoulli draws' coreset sizes equal the
  oracle's counts from the same lambda, the draws with replacement hold
  exactly s_out samples, and every draw meets (1 + eps) with f(x) summed by
  the oracle and the optimum bounded below by its weak-duality certificate.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import l1, philox, sampling

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


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def synthetic_lambda(n, seed):
    rng = np.random.default_rng(seed)
    lam = (rng.gamma(0.7, size=n) * rng.choice([1.0, 1e3], size=n, p=[0.999, 0.001])).astype(np.float32)
    lam[rng.choice(n, size=n // 10, replace=False)] = 0.0
    return lam


@pytest.mark.parametrize("n,s,draw", [(5, 7, 0), (1000, 300, 3), (1000003, 5000, 1), (1 << 24, 20000, 7)])
def test_replacement_draw_against_oracle(F, ctx, n, s, draw):
    lam = synthetic_lambda(n, n)
    seed = 77 + n
    print(f"with replacement n={n} s={s} draw={draw}", flush=True)
    idx, w, S = F.l1_select_draw(ctx, torch.from_numpy(lam).cuda(), None, s, seed, draw,
                                 F.FCT_SAMPLE_REPLACE, s)
    assert S == s
    gi, gw = host(idx)[:s], host(w)[:s]
    oi, ow = sampling.select_with_replacement(lam.astype(np.float64), s, seed, draw)
    assert np.all(lam[gi] > 0)
    bad = np.flatnonzero(gi != oi)
    if bad.size:
        # only ties at an interval end are allowed to differ
        C = np.cumsum(lam.astype(np.float64))
        u = (philox.replacement_words(seed, s, draw).astype(np.float64) + 0.5) * 2.0 ** -32
        t = u * C[-1]
        for j in bad:
            near = np.min(np.abs(C[max(0, oi[j] - 2):oi[j] + 2] - t[j]))
            assert near <= 1e-12 * C[-1], (j, gi[j], oi[j])
    assert bad.size <= max(1, s // 10000)
    ok = gi == oi
    assert np.allclose(gw[ok], ow[ok], rtol=1e-12)


@pytest.mark.parametrize("draw", [0, 1, 5])
def test_bernoulli_draw_against_oracle(F, ctx, draw):
    n = 300007
    lam = synthetic_lambda(n, 3)
    tot = torch.tensor([float(lam.astype(np.float64).sum())], dtype=torch.float64, device="cuda")
    s_out = 4000
    cap = 2 * s_out + 8 * int(np.sqrt(s_out)) + 1024
    idx, w, S = F.l1_select_draw(ctx, torch.from_numpy(lam).cuda(), tot, s_out, 19, draw,
                                 F.FCT_SAMPLE_BERNOULLI, cap)
    p = sampling.probabilities(lam, s_out, float(host(tot)[0]))
    oi, ow = sampling.select(p, 19, draw)
    assert S == oi.size
    assert np.array_equal(host(idx)[:S], oi)
    assert np.array_equal(host(w)[:S], ow)


@pytest.mark.parametrize("mode", ["bernoulli", "replace"])
def test_multi_draw_regression(F, ctx, mode):
    w = synth.scaled(synth.LARGE, 1 << 20)   # the deterministic owner sketch
    A, b, _ = synth.generate(w)
    Ad, bd = torch.from_numpy(A).cuda(), torch.from_numpy(b).cuda()
    K = 4
    md = F.FCT_SAMPLE_BERNOULLI if mode == "bernoulli" else F.FCT_SAMPLE_REPLACE
    prm = F.params(s=w.s, r1=w.r1, r2=w.r2, s_out=w.s_out, seed=w.seed)
    X, obj, S, status, st = F.l1_regress_multi(ctx, Ad, bd, prm, K, md, eps=w.eps)
    assert st == 0, status
    # the same sampling pass through the single calls: its lambda decides the draws
    _, R = F.fct_sketch(ctx, Ad, bd, w.s, w.r1, w.seed)
    lam, _, tot = F.l1_sample_probs(ctx, Ad, bd, R, w.r2, w.seed, w.s_out, want_p=False)
    lam_h = host(lam).astype(np.float64)
    if mode == "bernoulli":
        p = sampling.probabilities(lam_h, w.s_out, float(host(tot)[0]))
        for k in range(K):
            assert S[k] == int(np.count_nonzero(philox.sample_words(w.seed, w.n, k) < sampling.thresholds(p)))
    else:
        assert all(v == w.s_out for v in S)
    At, b64 = A.T, b.astype(np.float64)
    fs = [l1.objective(At, b64, X[k], chunk=1 << 18) for k in range(K)]
    x0, _ = F.l1_solve(ctx, Ad, bd, torch.ones(w.n, dtype=torch.float64, device="cuda"), iters=120)
    lower = l1.dual_lower_bound(At, b64, x0, threads=16, stop_at=max(fs) / (1 + 0.5 * w.eps))
    for k, f in enumerate(fs):
        print(f"{mode} draw {k}: S={S[k]} f/lower={f / lower:.6f}")
        assert f <= (1 + w.eps) * lower, (k, f / lower)
    assert len({tuple(np.round(x, 12)) for x in X}) == K   # independent draws, different solutions
