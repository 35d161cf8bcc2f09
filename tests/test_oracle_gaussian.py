"""Pins of the oracle's Gaussian Pi2 (the optimized regression figure, step 4)
and of the estimator it feeds.

* the stream-2 Box-Muller variates are standard normal (KS against the
  normal CDF, mean and variance), and the median of their absolute values is
  Phi^-1(3/4) (golden value: the median of the half-Gaussian in the proof of
  the optimized regression theorem);
* with Gaussian Pi2 the entries (U Pi2)_ij are N(0, ||U_(i)||_2^2), so for
  many columns lambda_i / ||U_(i)||_2 tends to Phi^-1(3/4) for every row;
* the probabilities are normalized (sum p <= s_out) and the whole optimized
  path is exact when every row is kept.
"""
import os

import numpy as np
import scipy.stats

from oracle import basis, fct, l1, philox, pipeline, sampling

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _median_abs_gaussian():
    with open(os.path.join(GOLDEN, "median_abs_gaussian.txt")) as fh:
        return float([ln for ln in fh if not ln.startswith("#")][0])


def test_gaussian_stream_is_standard_normal():
    g = philox.pi2_gaussian_matrix(11, 1000, 200).ravel()
    assert scipy.stats.kstest(g, "norm").pvalue > 1e-3
    assert abs(g.mean()) < 5.0 / np.sqrt(g.size)
    assert abs(g.var() - 1.0) < 5.0 * np.sqrt(2.0 / g.size)


def test_median_abs_gaussian_matches_golden():
    m = _median_abs_gaussian()
    assert abs(m - scipy.stats.norm.ppf(0.75)) < 1e-15
    g = philox.pi2_gaussian_matrix(3, 2000, 500).ravel()
    # the sample median of 10^6 half-normals is within a few 1e-3 of the median
    assert abs(np.median(np.abs(g)) - m) < 4e-3


def test_gaussian_and_cauchy_pi2_differ_and_use_stream_2():
    a = philox.pi2_gaussian_matrix(5, 4, 3)
    b = philox.pi2_matrix(5, 4, 3)
    w = philox.stream_words(5, philox.STREAM_PI2, np.arange(12, dtype=np.uint64))
    assert np.array_equal(b.ravel(), philox.cauchy_from_word(w[0]))
    assert np.array_equal(a.ravel(), philox.gaussian_from_words(w[0], w[1]))
    assert not np.allclose(a, b)


def test_lambda_tracks_row_l2_norm_with_gaussian_pi2():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((60, 6)) * np.array([1.0, 30.0, 0.01, 2.0, 5.0, 0.3])
    R = basis.qr_r(X)  # U = X R^-1 has orthonormal columns
    M = basis.m_matrix(R, 9, 4001, pi2="gaussian")
    lam = sampling.row_norm_estimates(X, M)
    U = X @ np.linalg.inv(R)
    ratio = lam / np.linalg.norm(U, axis=1)
    assert np.all(np.abs(ratio - _median_abs_gaussian()) < 0.06), ratio


def test_optimized_path_probabilities_and_all_rows_exact():
    rng = np.random.default_rng(4)
    n, d = 3000, 3
    A = rng.standard_normal((n, d))
    b = A @ rng.standard_normal(d) + rng.laplace(0, 0.1, n)
    out = pipeline.l1_regress(A, b, s=16, r1=64, r2=8, s_out=400, seed=2, pi2="gaussian")
    assert out["p"].sum() <= 400 * (1 + 1e-12)
    full = pipeline.l1_regress(A, b, s=16, r1=64, r2=8, s_out=1e30, seed=2, pi2="gaussian")
    assert full["idx"].size == n
    _, fopt = l1.lp(A, b)
    assert full["objective"] <= fopt * (1 + 1e-9)
