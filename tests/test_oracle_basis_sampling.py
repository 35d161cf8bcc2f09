"""Pins of the oracle's QR, M, row-norm estimator, probabilities and selection.

* R: R^T R = Y^T Y, Y R^-1 has orthonormal columns (the note in step 2 of the
  regression figure), R equals the Cholesky factor of Y^T Y (another library
  route), rank deficiency is detected;
* M: R M = Pi2 and Pi2 is Cauchy distributed;
* lambda: exact for one-hot rows (U_i is a scaled row of R^-1, so Lambda_i is
  a scaled row of M); the median lemma's bound on lambda_i / ||U_i||_1;
* probabilities: sum p <= s_out, p = 1 when s_out is huge;
* selection: thresholds at p = 0 and p = 1, E[S] = sum p, and the l1
  sampling lemma's unbiasedness E ||D U y||_1 = ||U y||_1.
"""
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.stats

from oracle import basis, fct, philox, sampling

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _sketch(n=4000, q=5, s=16, r1=40, seed=1):
    X = np.random.default_rng(seed).standard_normal((n, q)) * np.array([1, 10, 0.1, 3, 1])[:q]
    Y = fct.pi1_apply(X, s, r1, seed=seed)
    return X, Y


def test_qr_r_factor_properties():
    X, Y = _sketch()
    R = basis.qr_r(Y)
    assert np.allclose(np.tril(R, -1), 0)
    assert np.all(np.diag(R) > 0)
    assert np.allclose(R.T @ R, Y.T @ Y, rtol=1e-12, atol=1e-12 * np.abs(Y.T @ Y).max())
    Q = Y @ np.linalg.inv(R)
    assert np.allclose(Q.T @ Q, np.eye(R.shape[0]), atol=1e-10)
    L = scipy.linalg.cholesky(Y.T @ Y, lower=False)
    assert np.allclose(R, L, rtol=1e-8, atol=1e-8 * np.abs(R).max())


def test_rank_deficient_detected():
    X, Y = _sketch()
    Y[:, 2] = 2.0 * Y[:, 1]
    with pytest.raises(basis.RankDeficient):
        basis.qr_r(Y)


def test_m_solves_triangular_system():
    _, Y = _sketch()
    R = basis.qr_r(Y)
    M = basis.m_matrix(R, seed=5, r2=8)
    P2 = philox.pi2_matrix(5, R.shape[0], 8)
    assert np.allclose(R @ M, P2, rtol=1e-12, atol=1e-12 * np.abs(P2).max())
    big = philox.pi2_matrix(6, 40, 50).ravel()
    assert scipy.stats.kstest(big, lambda t: 0.5 + np.arctan(t) / np.pi).pvalue > 1e-4


def test_lambda_one_hot_rows_closed_form():
    q, r2 = 4, 6
    R = np.triu(np.random.default_rng(2).standard_normal((q, q))) + 3 * np.eye(q)
    M = basis.m_matrix(R, seed=3, r2=r2)
    X = np.zeros((q, q))
    X[np.arange(q), np.arange(q)] = np.array([1.0, -2.0, 0.5, 4.0])
    lam = sampling.row_norm_estimates(X, M)
    for a in range(q):
        v = np.sort(np.abs(X[a, a] * M[a]))
        assert np.isclose(lam[a], 0.5 * (v[r2 // 2 - 1] + v[r2 // 2]), rtol=1e-14)


def _prob_median_in_range(r2: int) -> float:
    """Exact P(1/2 <= median of r2 |Cauchy| <= 3/2) for odd r2 (binomial order statistic)."""
    F = lambda x: 2.0 / np.pi * np.arctan(x)          # CDF of |Cauchy|
    k = (r2 + 1) // 2                                  # the median is the k-th order statistic
    below = lambda x: scipy.stats.binom.sf(k - 1, r2, F(x))   # P(at least k samples <= x)
    return below(1.5) - below(0.5)


def test_median_lemma_rate():
    c, inv = np.loadtxt(os.path.join(GOLDEN, "median_cauchy_constant.txt"))
    r2 = 101
    exact = _prob_median_in_range(r2)
    # Reading: the lemma's printed constant c = 2 arctan(1/5)^2 ~ 0.078 omits the
    # factor (2/pi)^2 of the Hoeffding argument (|C| <= 3/2 has probability
    # 1/2 + (2/pi) arctan(1/5)); the exact tail at r2 = 101 exceeds 2 exp(-0.07 r2).
    assert 1 - exact > 2 * np.exp(-c * r2)
    assert 1 - exact <= 2 * np.exp(-2 * (2 / np.pi * np.arctan(0.2)) ** 2 * r2)
    X, _ = _sketch(n=2000)
    fracs = []
    for seed in range(12):
        Y = fct.pi1_apply(X, 16, 40, seed=seed)
        R = basis.qr_r(Y)
        M = basis.m_matrix(R, seed=seed, r2=r2)
        ratio = sampling.row_norm_estimates(X, M) / sampling.exact_l1_leverage(X, R)
        fracs.append(np.mean((ratio >= 0.5) & (ratio <= 1.5)))
    # rows of one draw share Pi2, so the draws (not the rows) are the samples
    assert np.mean(fracs) >= exact - 4 * np.std(fracs) / np.sqrt(len(fracs)) - 0.002
    assert inv == 15 and 1 / c <= inv + 1e-12


def test_probabilities():
    lam = np.random.default_rng(1).exponential(size=1000)
    p = sampling.probabilities(lam, 100)
    assert np.all((p > 0) & (p <= 1)) and p.sum() <= 100 + 1e-9
    assert np.all(sampling.probabilities(lam, 1e30) == 1.0)


def test_selection_thresholds_and_mean():
    p = np.array([0.0, 1.0, 1.0, 0.0])
    idx, w = sampling.select(p, seed=1)
    assert list(idx) == [1, 2] and np.all(w == 1.0)
    assert sampling.thresholds(np.array([1.0]))[0] == 2**32
    p = np.full(20000, 0.3)
    counts = [sampling.select(p, seed=s)[0].size for s in range(5)]
    assert abs(np.mean(counts) - 6000) < 4 * np.sqrt(20000 * 0.3 * 0.7)


def test_l1_sampling_lemma_unbiased():
    # E ||D U y||_1 = ||U y||_1 for the Bernoulli D with D_ii = 1/p_i
    g = np.random.default_rng(3)
    U = g.standard_normal((400, 3)) * g.exponential(size=(400, 1))
    y = g.standard_normal(3)
    lam = np.abs(U).sum(axis=1)
    p = sampling.probabilities(lam, 60)
    vals = []
    for sd in range(300):
        idx, w = sampling.select(p, seed=sd)
        vals.append(np.sum(w * np.abs(U[idx] @ y)))
    vals = np.array(vals)
    target = np.abs(U @ y).sum()
    assert abs(vals.mean() - target) < 4 * vals.std() / np.sqrt(len(vals))
