"""GPU parity at the full sizes of the benchmark workloads against the oracle.

* The whole sketch Y = Pi1 [A, -b] of tall (4,194,304 x 32), precision
  (33,554,432 x 64) and large (268,435,456 x 16), element by element against
  the oracle's, stored in tests/golden/ by make_full_sketches.py (oracle and
  synth only), gated at 1e-5 of each row's l1 mass; R against the oracle's
  Gram matrix of that sketch.  The same for the FCT2 sketch of each workload
  (block sizes from the generator's table).
* lambda on sampled rows for the FP32 and BF16 passes (the oracle evaluates
  those rows from the GPU's R), and the selection given the GPU's lambda
  (over all rows, or a window of rows).
* The (1 + eps) objective of the plain and BF16 regressions (and, on tall
  and large, of the optimized regression with Gaussian Pi2): f(x) is the
  oracle's FP64 host sum, and the optimum is bounded below by the oracle's
  weak-duality certificate.

The oracle never sees the GPU's outputs as expected values: it recomputes
each checked quantity from the same input bytes (and, for lambda and the
selection, from the GPU's R or lambda where the check is of the next step).
"""
import os

import numpy as np
import pytest
import torch

import synth
from oracle import basis, l1, lowp, philox, sampling

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

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


def check_one_plus_eps(F, ctx, L, optimized=False):
    """(1 + eps) of the plain and BF16 regressions, and with ``optimized`` of
    the optimized regression (Gaussian Pi2, r2 = 8)."""
    w = L.w
    prm = F.params(s=w.s, r1=w.r1, r2=w.r2, s_out=w.s_out, seed=w.seed)
    xs = {"plain": F.l1_regress(ctx, L.Ad, L.bd, prm, eps=w.eps)[0],
          "bf16": F.l1_regress(ctx, L.Ad, L.bd, prm, eps=w.eps, A_lowp=L.Al, b_lowp=L.bl)[0]}
    if optimized:
        po = F.params(s=w.s, r1=w.r1, r2=8, s_out=w.s_out, seed=w.seed,
                      flags=F.FCT_FLAG_GAUSSIAN_PI2)
        xs["optimized"] = F.l1_regress(ctx, L.Ad, L.bd, po, eps=w.eps)[0]
    # f(x) by the oracle: an FP64 host sum over the input bytes
    fs = {name: l1.objective(L.A.T, L.b, x, chunk=1 << 22) for name, x in xs.items()}
    print(f"{w.name}: regressions done {fs}", flush=True)
    # a candidate optimum from the all-rows solver; the oracle's dual bound is
    # valid whoever produced the candidate
    x0, _ = F.l1_solve(ctx, L.Ad, L.bd, torch.ones(w.n, dtype=torch.float64, device="cuda"), iters=120)
    need = max(fs.values()) / (1 + 0.5 * w.eps)   # a bound this high settles both claims
    lower = l1.dual_lower_bound(L.A.T, L.b, x0, threads=16, stop_at=need)
    print(f"{w.name}: lower bound {lower}", flush=True)
    assert lower > 0
    for name, f in fs.items():
        print(f"{w.name} {name}: f / lower bound = {f / lower:.9f}")
        assert f <= (1 + w.eps) * lower, (name, f / lower)


def check_whole_sketch(F, ctx, L):
    """The whole sketch against the oracle's, and R against the oracle's
    Gram matrix of it."""
    w = L.w
    Yo = np.load(os.path.join(GOLDEN, f"sketch_{w.name}.npy"))
    S = np.load(os.path.join(GOLDEN, f"scale_{w.name}.npy"))
    Y, R = F.fct_sketch(ctx, L.Ad, L.bd, w.s, w.r1, w.seed)
    Yg = host(Y).astype(np.float64)
    err = np.max(np.abs(Yg - Yo), axis=1)
    print(f"{w.name}: whole sketch max err / S = {float(np.max(err / S)):.3e}", flush=True)
    assert np.all(err <= 1e-5 * S), float(np.max(err / S))
    # R^T R = Y^T Y for the FP64 sketch R was taken from, which is within
    # 1e-5 S_i of the oracle's row by row: |d(Y^T Y)_jk| <= 1e-5 sum_i S_i
    # (|Y_ij| + |Y_ik|) + (1e-5)^2 sum_i S_i^2, plus the QR's rounding
    Rg = host(R)
    assert np.all(np.diag(Rg) > 0) and np.allclose(np.tril(Rg, -1), 0)
    G = Yo.T @ Yo
    aY = S[:, None] * np.abs(Yo)
    bound = 1e-5 * (aY.sum(axis=0)[:, None] + aY.sum(axis=0)[None, :]) + 1e-10 * float(S @ S)
    bound += 1e-12 * np.abs(G).max()
    assert np.all(np.abs(Rg.T @ Rg - G) <= bound), float(np.max(np.abs(Rg.T @ Rg - G) / bound))
    return R


def fct2_params(name):
    """(t, s) of the stored FCT2 sketch of a workload (the generator's table)."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_full_sketches",
                                                  os.path.join(GOLDEN, "make_full_sketches.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.FCT2_PARAMS[name]


def check_fct2_whole_sketch(F, ctx, L, name):
    """FCT2's whole sketch against the oracle's (stored by the generator)."""
    w = L.w
    t, s = fct2_params(name)
    Yo = np.load(os.path.join(GOLDEN, f"fct2_sketch_{w.name}.npy"))
    S = np.load(os.path.join(GOLDEN, f"fct2_scale_{w.name}.npy"))
    Y, R = F.fct2_sketch(ctx, L.Ad, L.bd, t, s, w.r1, w.seed)
    Yg = host(Y).astype(np.float64)
    err = np.max(np.abs(Yg - Yo), axis=1)
    print(f"{w.name}: FCT2 (t={t}, s={s}) whole sketch max err / S = {float(np.max(err / S)):.3e}",
          flush=True)
    assert np.all(err <= 1e-5 * S), float(np.max(err / S))
    Rg = host(R)
    assert np.all(np.diag(Rg) > 0) and np.allclose(np.tril(Rg, -1), 0)


# ---- tall ------------------------------------------------------------------

@pytest.fixture(scope="module")
def tall(F, ctx):
    L = Loaded(F, ctx, synth.TALL)
    yield L
    L.close()


def test_tall_full_size_sketch_lambda_selection(F, ctx, tall):
    R = check_whole_sketch(F, ctx, tall)
    lam, tot = check_lambda_sampled(F, ctx, tall, R, np.random.default_rng(1))
    check_selection(F, ctx, tall, lam, tot)


def test_tall_full_size_fct2_sketch(F, ctx, tall):
    check_fct2_whole_sketch(F, ctx, tall, "tall")


def test_tall_full_size_one_plus_eps(F, ctx, tall):
    check_one_plus_eps(F, ctx, tall, optimized=True)


# ---- precision and large ---------------------------------------------------

@pytest.fixture(scope="module")
def precision(F, ctx):
    L = Loaded(F, ctx, synth.PRECISION)
    yield L
    L.close()


def test_precision_full_size_sketch_lambda_selection(F, ctx, precision):
    R = check_whole_sketch(F, ctx, precision)
    lam, tot = check_lambda_sampled(F, ctx, precision, R, np.random.default_rng(2))
    check_selection(F, ctx, precision, lam, tot, window=(1 << 24, (1 << 24) + (1 << 22)))


def test_precision_full_size_fct2_sketch(F, ctx, precision):
    check_fct2_whole_sketch(F, ctx, precision, "precision")


def test_precision_full_size_one_plus_eps(F, ctx, precision):
    check_one_plus_eps(F, ctx, precision)


@pytest.fixture(scope="module")
def large(F, ctx):
    L = Loaded(F, ctx, synth.LARGE)
    yield L
    L.close()


def test_large_full_size_sketch_lambda_selection(F, ctx, large):
    R = check_whole_sketch(F, ctx, large)
    lam, tot = check_lambda_sampled(F, ctx, large, R, np.random.default_rng(3))
    check_selection(F, ctx, large, lam, tot, window=(3 << 26, (3 << 26) + (1 << 22)))


def test_large_full_size_fct2_sketch(F, ctx, large):
    check_fct2_whole_sketch(F, ctx, large, "large")


def test_large_full_size_one_plus_eps(F, ctx, large):
    check_one_plus_eps(F, ctx, large, optimized=True)
