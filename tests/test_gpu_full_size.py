"""GPU parity at the full sizes of the benchmark workloads, on outputs the
oracle can compute piece by piece.

* tall (4,194,304 x 32 FP32; the benchmark's workload): lambda on sampled
  rows for the FP32 and BF16 passes, the selection over all rows given the
  GPU's lambda, and the (1 + eps) objective of both paths against a
  weak-duality lower bound.
* precision (33,554,432 x 64 FP32 + BF16 copy) and large (268,435,456 x 16
  FP32): the sketch of one window of rows against the oracle (the streams
  are indexed by global row), the whole sketch against the sum of window
  sketches, R against the sketch it factors, sampled lambda, the selection
  in a window of rows, and the (1 + eps) objective.

The oracle never sees the GPU's outputs as expected values: it recomputes
each checked quantity from the same input bytes (and, for lambda and the
selection, from the GPU's R or lambda where the check is of the next step).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import basis, fct, l1, lowp, philox, sampling

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


class Loaded:
    """One workload: host arrays, device copies and its BF16 copies."""

    def __init__(self, F, ctx, w):
        self.w = w
        self.A, self.b, _ = synth.generate(w, threads=16)
        self.Ad = torch.from_numpy(self.A).cuda()
        self.bd = torch.from_numpy(self.b).cuda()
        self.Al = F.fct_to_bf16(ctx, self.Ad)
        self.bl = F.fct_to_bf16(ctx, self.bd)
        torch.cuda.synchronize()

    def rows(self, idx):
        """X = [A, -b] at the given rows, FP64."""
        return np.hstack([self.A[:, idx].T.astype(np.float64), -self.b[idx].astype(np.float64)[:, None]])

    def close(self):
        del self.Ad, self.bd, self.Al, self.bl
        torch.cuda.empty_cache()


def check_lambda_sampled(F, ctx, L, R, rng):
    w = L.w
    n = w.n
    idx = np.sort(rng.choice(n, size=4096, replace=False))
    M = basis.m_matrix(host(R), w.seed, w.r2)
    X = L.rows(idx)
    lam, _, tot = F.l1_sample_probs(ctx, L.Ad, L.bd, R, w.r2, w.seed, w.s_out, want_p=False)
    lam_h = host(lam)
    ref = sampling.row_norm_estimates(X, M)
    scale = (np.abs(X) @ np.abs(M)).max(axis=1)
    assert np.all(np.abs(lam_h[idx] - ref) <= 1e-5 * scale), "FP32 lambda"
    # BF16 pass: the same formula on the BF16-rounded X and M
    lam_b, _, _ = F.l1_sample_probs(ctx, L.Al, L.bl, R, w.r2, w.seed, w.s_out, want_p=False)
    Xl = lowp.round_bf16(X.astype(np.float32))
    Ml = lowp.round_bf16(M.astype(np.float32))
    ref_b = sampling.row_norm_estimates(Xl, Ml)
    scale_b = (np.abs(Xl) @ np.abs(Ml)).max(axis=1)
    assert np.all(np.abs(host(lam_b)[idx] - ref_b) <= 1e-5 * scale_b), "BF16 lambda"
    assert np.isclose(host(tot)[0], lam_h.astype(np.float64).sum(), rtol=1e-10)
    return lam, tot


def check_selection(F, ctx, L, lam, tot, window=None):
    w = L.w
    n = w.n
    cap = 2 * w.s_out + 8 * int(np.sqrt(w.s_out)) + 1024
    idx, wt, S = F.l1_select(ctx, lam, tot, w.s_out, w.seed, cap)
    gi, gw = host(idx)[:S], host(wt)[:S]
    lam_h = host(lam).astype(np.float64)
    total = float(host(tot)[0])
    lo, hi = (0, n) if window is None else window
    p = sampling.probabilities(lam_h[lo:hi], w.s_out, total)
    keep = philox.sample_words(w.seed, hi - lo, start=lo) < sampling.thresholds(p)
    oidx = lo + np.flatnonzero(keep)
    sel = (gi >= lo) & (gi < hi)
    assert np.array_equal(gi[sel], oidx)
    assert np.array_equal(gw[sel], 1.0 / p[oidx - lo])


def check_one_plus_eps(F, ctx, L):
    w = L.w
    prm = F.params(s=w.s, r1=w.r1, r2=w.r2, s_out=w.s_out, seed=w.seed)
    x_plain, _, _ = F.l1_regress(ctx, L.Ad, L.bd, prm, eps=w.eps)
    x_bf16, _, _ = F.l1_regress(ctx, L.Ad, L.bd, prm, eps=w.eps, A_lowp=L.Al, b_lowp=L.bl)
    fs = {name: float(F.fct_l1_objective(ctx, L.Ad, L.bd, x))
          for name, x in (("plain", x_plain), ("bf16", x_bf16))}
    print(f"{w.name}: regressions done {fs}", flush=True)
    # a candidate optimum from the all-rows solver; the oracle's dual bound is
    # valid whoever produced the candidate
    x0, _ = F.l1_solve(ctx, L.Ad, L.bd, torch.ones(w.n, dtype=torch.float64, device="cuda"), iters=120)
    f0 = float(F.fct_l1_objective(ctx, L.Ad, L.bd, x0))
    print(f"{w.name}: all-rows candidate {f0}", flush=True)
    need = max(fs.values()) / (1 + 0.5 * w.eps)   # a bound this high settles both claims
    lower = l1.dual_lower_bound(L.A.T, L.b, x0, threads=16, stop_at=need)
    print(f"{w.name}: all-rows candidate f / lower bound = {f0 / lower:.9f}", flush=True)
    assert lower > 0
    for name, f in fs.items():
        print(f"{w.name} {name}: f / lower bound = {f / lower:.9f}")
        assert f <= (1 + w.eps) * lower, (name, f / lower)


# ---- tall ------------------------------------------------------------------

@pytest.fixture(scope="module")
def tall(F, ctx):
    L = Loaded(F, ctx, synth.TALL)
    yield L
    L.close()


def test_tall_full_size_lambda_and_selection(F, ctx, tall):
    w = tall.w
    _, R = F.fct_sketch(ctx, tall.Ad, tall.bd, w.s, w.r1, w.seed, want_y=False)
    lam, tot = check_lambda_sampled(F, ctx, tall, R, np.random.default_rng(1))
    check_selection(F, ctx, tall, lam, tot)


def test_tall_full_size_one_plus_eps(F, ctx, tall):
    check_one_plus_eps(F, ctx, tall)


# ---- precision and large ---------------------------------------------------

def check_windows_and_basis(F, ctx, L, win_rows, oracle_row0):
    """Window sketch vs the oracle, the whole sketch vs the sum of windows, R vs Y."""
    w = L.w
    n = w.n
    q = w.d + 1
    Y, R = F.fct_sketch(ctx, L.Ad, L.bd, w.s, w.r1, w.seed)
    Yg = host(Y).astype(np.float64)
    total = np.zeros_like(Yg)
    absum = np.zeros_like(Yg)
    starts = list(range(0, n, win_rows))
    for a in starts:
        bnd = min(n, a + win_rows)
        Yw = host(F.fct_sketch_window(ctx, L.Ad[:, a:bnd], L.bd[a:bnd], w.s, w.r1, w.seed, a)).astype(np.float64)
        total += Yw
        absum += np.abs(Yw)
    # one window of 2^20 rows inside the design against the oracle
    a, bnd = oracle_row0, oracle_row0 + (1 << 20)
    Yw = host(F.fct_sketch_window(ctx, L.Ad[:, a:bnd], L.bd[a:bnd], w.s, w.r1, w.seed, a)).astype(np.float64)
    Yo, S = fct.pi1_apply(L.rows(np.arange(a, bnd)), w.s, w.r1, w.seed, return_scale=True, row0=a)
    err = np.max(np.abs(Yw - Yo), axis=1)
    assert np.all(err <= 1e-5 * S), float(np.max(err / S))
    # partial sums are rounded to FP32 once per row range: a few ulp of the
    # summed magnitudes
    assert np.all(np.abs(Yg - total) <= 1e-5 * absum.max(axis=1, keepdims=True))
    # R factors the sketch: R^T R = Y^T Y (Y here is the FP32 rounding of the
    # FP64 sketch R was computed from)
    Rg = host(R)
    G = Yg.T @ Yg
    assert np.all(np.diag(Rg) > 0) and np.allclose(np.tril(Rg, -1), 0)
    assert np.max(np.abs(Rg.T @ Rg - G)) <= 1e-5 * np.abs(G).max()
    return R


@pytest.fixture(scope="module")
def precision(F, ctx):
    L = Loaded(F, ctx, synth.PRECISION)
    yield L
    L.close()


def test_precision_full_size_sketch_lambda_selection(F, ctx, precision):
    R = check_windows_and_basis(F, ctx, precision, 1 << 23, 5 << 22)
    lam, tot = check_lambda_sampled(F, ctx, precision, R, np.random.default_rng(2))
    check_selection(F, ctx, precision, lam, tot, window=(1 << 24, (1 << 24) + (1 << 22)))


def test_precision_full_size_one_plus_eps(F, ctx, precision):
    check_one_plus_eps(F, ctx, precision)


@pytest.fixture(scope="module")
def large(F, ctx):
    L = Loaded(F, ctx, synth.LARGE)
    yield L
    L.close()


def test_large_full_size_sketch_lambda_selection(F, ctx, large):
    R = check_windows_and_basis(F, ctx, large, 1 << 26, 37 << 22)
    lam, tot = check_lambda_sampled(F, ctx, large, R, np.random.default_rng(3))
    check_selection(F, ctx, large, lam, tot, window=(3 << 26, (3 << 26) + (1 << 22)))


def test_large_full_size_one_plus_eps(F, ctx, large):
    check_one_plus_eps(F, ctx, large)
