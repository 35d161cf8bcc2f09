"""Pins of the oracle's FCT2 (section "FCT2 Construction"): the fast form
against Pi1 built entry by entry, the Johnson-Lindenstrauss property of the
block G, the 1-stability of C, the embedding's lower bound with the paper's
scale, and windows that add up to the whole."""
import numpy as np
from scipy import stats

from oracle import fct, philox


def test_fast_equals_dense_definition():
    rng = np.random.default_rng(0)
    for n, t, s, r1 in [(300, 64, 8, 32), (129, 32, 32, 7), (64, 64, 3, 50), (1000, 16, 4, 9)]:
        X = rng.standard_normal((n, 3))
        Y = fct.fct2_apply(X, t, s, r1, seed=n)
        P = fct.fct2_dense(n, t, s, r1, seed=n)
        assert np.allclose(Y, P @ X, rtol=1e-12, atol=1e-12 * np.abs(Y).max())


def test_g_preserves_squared_norm_in_expectation():
    """E ||G z||_2^2 = ||z||_2^2 for G = sqrt(t/s) P H_t D (rows of P uniform)."""
    rng = np.random.default_rng(1)
    t, s = 64, 8
    z = rng.standard_normal(t) * rng.gamma(0.5, size=t)
    ratios = []
    for seed in range(3000):
        hz = fct.fwht_blocks((z * philox.signs(seed, t))[None, :, None])[0, :, 0]
        rows = philox.fct2_rows(seed, 1, s, t)[0]
        ratios.append(np.sum((np.sqrt(t / s) * hz[rows]) ** 2) / np.sum(z ** 2))
    assert abs(np.mean(ratios) - 1.0) < 0.05


def test_rows_of_c_times_z_are_cauchy():
    """For one column, Y_i / c is Cauchy with scale ||Z||_1 (1-stability)."""
    rng = np.random.default_rng(2)
    n, t, s, r1 = 2048, 64, 8, 4001
    x = rng.standard_normal((n, 1))
    Y = fct.fct2_apply(x, t, s, r1, seed=3)[:, 0]
    # Z of the same transform, from the definition
    D = philox.signs(3, n)
    hz = fct.fwht_blocks((x[:, 0] * D).reshape(n // t, t, 1))[:, :, 0]
    rows = philox.fct2_rows(3, n // t, s, t)
    Z = np.sqrt(t / s) * hz[np.arange(n // t)[:, None], rows]
    u = Y / (fct.fct2_scale(r1, s, t) * np.abs(Z).sum())
    assert stats.kstest(u, "cauchy").pvalue > 1e-3


def test_lower_bound_of_the_embedding():
    """||A x||_1 <= ||Pi1 A x||_1 for the x tried (Theorem FCT, the scale
    8/r1 sqrt(pi t/(2 s)) is what makes the lower bound hold)."""
    rng = np.random.default_rng(4)
    n, d, t, s, r1 = 4096, 4, 64, 16, 64
    A = rng.standard_normal((n, d)) * rng.gamma(0.7, size=(n, 1))
    PA = fct.fct2_apply(A, t, s, r1, seed=11)
    ratios = [np.abs(PA @ x).sum() / np.abs(A @ x).sum() for x in rng.standard_normal((200, d))]
    assert min(ratios) >= 1.0, min(ratios)


def test_windows_add_up_to_the_whole():
    rng = np.random.default_rng(5)
    X = rng.standard_normal((700, 2))
    t = 64
    whole = fct.fct2_apply(X, t, 8, 16, seed=9)
    parts = fct.fct2_apply(X[:320], t, 8, 16, seed=9) + fct.fct2_apply(X[320:], t, 8, 16, seed=9, row0=320)
    assert np.allclose(whole, parts, rtol=1e-12, atol=1e-12 * np.abs(whole).max())
