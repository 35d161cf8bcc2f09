"""Pins of the oracle's exact l1 optima and the whole oracle path (CPU only).

* brute force over interpolating subsets == HiGHS LP (two independent
  routes), weighted and unweighted;
* one column of ones: the optimum is the median of b (closed form);
* canonical-row design: LP == per-coordinate weighted median;
* the vertex certificate accepts the LP optimum and its dual bound is valid;
* the oracle path: with every p_i = 1 the coreset is the whole problem and
  the answer is the exact optimum; on a scaled-down workload the objective
  is within (1 + eps) of the optimum (Theorem FCRsimp).
"""
import numpy as np
import pytest

import synth
from oracle import l1, lowp, pipeline


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("weighted", [False, True])
def test_brute_force_equals_lp(d, weighted):
    g = np.random.default_rng(10 * d + weighted)
    for _ in range(4):
        n = int(g.integers(d + 2, 15))
        A = g.standard_normal((n, d))
        b = A @ g.standard_normal(d) + g.standard_cauchy(n)
        w = g.uniform(0.5, 3.0, n) if weighted else None
        xb, fb = l1.brute_force(A, b, w)
        xl, fl = l1.lp(A, b, w)
        assert np.isclose(fb, fl, rtol=1e-9, atol=1e-9)


def test_median_closed_form():
    b = np.random.default_rng(1).standard_normal(101)
    x, f = l1.lp(np.ones((101, 1)), b)
    assert np.isclose(x[0], np.median(b), atol=1e-9)
    assert np.isclose(l1.weighted_median(b), np.median(b))


def test_separable_design_closed_form():
    A, b, coord, _ = synth.separable(3000, 4, seed=2, dtype=np.float64)
    w = np.random.default_rng(3).uniform(0.5, 2.0, 3000)
    xs = l1.separable_optimum(coord, b, 4, w)
    xl, fl = l1.lp(A.T, b, w)
    assert np.isclose(l1.objective(A.T, b, xs, w), fl, rtol=1e-10)


def test_vertex_certificate():
    g = np.random.default_rng(4)
    A = g.standard_normal((300, 4))
    b = A @ g.standard_normal(4) + g.laplace(size=300)
    xl, fl = l1.lp(A, b)
    xv, fv, ok, lower = l1.certify_vertex(A, b, xl)
    assert ok and np.isclose(fv, fl, rtol=1e-10) and lower <= fl * (1 + 1e-9)
    # a poor starting point: the bound stays a valid lower bound
    xv2, fv2, ok2, lower2 = l1.certify_vertex(A, b, xl + 0.5)
    assert lower2 <= fl * (1 + 1e-9)


def test_dual_lower_bound_valid_and_tight():
    g = np.random.default_rng(6)
    A = g.standard_normal((400, 5)) * 10.0 ** g.uniform(-3, 3, 5)
    A[::97] *= 1e4
    b = A @ g.standard_normal(5) + g.laplace(size=400) + 1e3 * g.standard_cauchy(400) * (g.random(400) < 0.02)
    w = g.uniform(0.5, 3.0, 400)
    xl, fl = l1.lp(A, b, w)
    lb = l1.dual_lower_bound(A, b, xl, w)
    assert lb <= fl * (1 + 1e-9) and lb >= fl * (1 - 1e-6)
    # from a poor candidate the bound stays below the optimum
    for xc in (np.zeros(5), xl * 1.1, g.standard_normal(5)):
        assert l1.dual_lower_bound(A, b, xc, w) <= fl * (1 + 1e-9)


def test_oracle_path_all_rows_is_exact():
    w = synth.scaled(synth.SMALL, 3000, d=3)
    A, b, _ = synth.generate(w)
    out = pipeline.l1_regress(A.T, b, s=16, r1=24, r2=8, s_out=1e30, seed=0)
    assert out["idx"].size == 3000
    _, fopt = l1.lp(A.T.astype(np.float64), b.astype(np.float64))
    assert np.isclose(out["objective"], fopt, rtol=1e-9)


def test_oracle_path_one_plus_eps():
    w = synth.scaled(synth.TALL, 20000, d=4, s_out=2500)
    A, b, _ = synth.generate(w)
    At, b64 = A.T.astype(np.float64), b.astype(np.float64)
    _, fopt = l1.lp(At, b64)
    out = pipeline.l1_regress(At, b64, s=64, r1=64, r2=16, s_out=2500, seed=0)
    assert out["objective"] <= (1 + 0.05) * fopt
    # the BF16 reading of the sampling pass is exercised too
    out_l = pipeline.l1_regress(A.T, b, s=64, r1=64, r2=16, s_out=2500, seed=0, lowp_pass2=True)
    assert out_l["objective"] <= (1 + 0.1) * fopt


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    g = np.random.default_rng(5)
    x = np.concatenate([g.standard_normal(10000) * 10.0 ** g.uniform(-20, 20, 10000),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38])]).astype(np.float32)
    ours = lowp.f32_to_bf16_bits(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)


def test_dual_lower_bound_chunked_rank_taus():
    # the large-n mode (FP64 products over row chunks, tau only at the ranks
    # just above the d smallest residuals) is still a valid and tight bound
    g = np.random.default_rng(9)
    A = (g.standard_normal((5000, 6)) * 10.0 ** g.uniform(-2, 2, 6)).astype(np.float32)
    b = A.astype(np.float64) @ g.standard_normal(6) + g.laplace(size=5000)
    xl, fl = l1.lp(A.astype(np.float64), b)
    lb = l1.dual_lower_bound(A, b, xl, rank_taus_only=True, chunk=777)
    assert lb <= fl * (1 + 1e-9) and lb >= fl * (1 - 1e-6)
    assert l1.dual_lower_bound(A, b, np.zeros(6), rank_taus_only=True, chunk=777) <= fl * (1 + 1e-9)
