"""Pins of the oracle's sampling with replacement and of several draws from
one sampling pass (the FastCauchyRegression figure's caption; the large-scale
evaluation's simultaneous solutions)."""
from fractions import Fraction

import numpy as np

import synth
from oracle import l1, philox, pipeline, sampling


def test_inversion_by_exact_interval_search():
    """Each sample's row from the definition, in exact rational arithmetic:
    the row whose interval [C_(i-1), C_i) of the running sums holds u * C_n."""
    lam = np.array([1.0, 3.0, 0.0, 4.0, 0.5, 2.5])
    rows, w = sampling.select_with_replacement(lam, 64, seed=5, instance=2)
    words = philox.replacement_words(5, 64, instance=2)
    C = [Fraction(0)]
    for v in lam:
        C.append(C[-1] + Fraction(v))
    for j in range(64):
        t = (Fraction(int(words[j])) + Fraction(1, 2)) / 2 ** 32 * C[-1]
        i = next(k for k in range(len(lam)) if C[k] <= t < C[k + 1])
        assert rows[j] == i
        assert np.isclose(w[j], float(C[-1] / (64 * Fraction(lam[i]))), rtol=1e-15)
    assert 2 not in rows  # a zero estimate is never drawn


def test_frequencies_follow_the_estimates():
    """Chi-square over many samples: the share of row i is lambda_i / sum."""
    from scipy import stats
    rng = np.random.default_rng(3)
    lam = rng.gamma(2.0, size=40)
    rows, _ = sampling.select_with_replacement(lam, 200000, seed=11)
    counts = np.bincount(rows, minlength=40)
    expected = 200000 * lam / lam.sum()
    assert stats.chisquare(counts, expected).pvalue > 1e-3


def test_weighted_sample_is_unbiased():
    """E sum_j w_j |r_(row_j)| = sum_i |r_i| for any fixed residual r."""
    rng = np.random.default_rng(7)
    lam = rng.gamma(1.5, size=500)
    r = rng.standard_normal(500) * rng.gamma(1.0, size=500)
    est = [np.sum(w * np.abs(r[rows])) for rows, w in
           (sampling.select_with_replacement(lam, 50, seed=9, instance=k) for k in range(4000))]
    assert abs(np.mean(est) / np.abs(r).sum() - 1) < 0.02


def test_draws_are_independent_streams():
    """Draw k uses instance k: draws differ, and draw 0 is the single draw."""
    lam = np.ones(10000)
    a = sampling.select_with_replacement(lam, 100, seed=1, instance=0)[0]
    b = sampling.select_with_replacement(lam, 100, seed=1, instance=1)[0]
    assert not np.array_equal(a, b)
    p = sampling.probabilities(lam, 100)
    s0 = sampling.select(p, 1, 0)[0]
    s1 = sampling.select(p, 1, 1)[0]
    assert not np.array_equal(s0, s1) and abs(s0.size - s1.size) < 60


def test_with_replacement_regression_meets_one_plus_eps():
    """Every draw of the with-replacement path, and of the Bernoulli path,
    meets (1 + eps) against the LP optimum on a small scaled workload."""
    w = synth.scaled(synth.SMALL, 12000, d=6)
    A, b, _ = synth.generate(w)
    At = A.T.astype(np.float64)
    _, fopt = l1.lp(At, b.astype(np.float64))
    for mode in ("replace", "bernoulli"):
        out = pipeline.l1_regress(At, b, s=64, r1=256, r2=8, s_out=600, seed=4,
                                  sampling_mode=mode, draws=3)
        for dr in out["draws"]:
            assert dr["objective"] <= 1.1 * fopt, (mode, dr["objective"] / fopt)
        if mode == "replace":
            assert all(dr["idx"].size == 600 for dr in out["draws"])
