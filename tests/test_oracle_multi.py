"""Pins of the oracle's multiple l1 regression and l1 subspace approximation
(sections "Generalizing to Multiple l1 Regression" and "Application to l1
norm Subspace Approximation")."""
import itertools

import numpy as np

import synth
from oracle import l1, pipeline


def test_one_right_hand_side_is_the_simple_regression():
    w = synth.scaled(synth.SMALL, 6000, d=5)
    A, b, _ = synth.generate(w)
    At = A.T.astype(np.float64)
    one = pipeline.l1_regress(At, b, s=64, r1=128, r2=8, s_out=500, seed=3)
    many = pipeline.l1_regress_mrhs(At, b[:, None], s=64, r1=128, r2=8, s_out=500, seed=3)
    assert np.array_equal(one["lam"], many["lam"])
    assert np.array_equal(one["idx"], many["idx"])
    assert np.allclose(many["W"][:, 0], one["x"], rtol=1e-9, atol=1e-9)


def test_every_column_within_one_plus_eps():
    rng = np.random.default_rng(5)
    n, d, k = 5000, 4, 3
    A = rng.standard_normal((n, d)) * np.array([1.0, 10.0, 0.1, 3.0])
    B = A @ rng.standard_normal((d, k)) + rng.laplace(0, 0.2, (n, k))
    B[rng.choice(n, 50, replace=False)] += 1e3 * rng.standard_cauchy((50, k))
    out = pipeline.l1_regress_mrhs(A, B, s=64, r1=256, r2=16, s_out=800, seed=9)
    for j in range(k):
        _, fopt = l1.lp(A, B[:, j])
        assert out["objective"][j] <= 1.1 * fopt, (j, out["objective"][j] / fopt)


def test_subspace_with_all_rows_is_the_best_hyperplane_fit():
    """Every row kept: each constrained regression is exact, and err_(j*) is
    the optimum of the reduction, which matches a brute-force search over the
    hyperplanes through d - 1 of the points (l1 fits interpolate)."""
    rng = np.random.default_rng(2)
    n, d = 9, 3
    A = rng.standard_normal((n, d))
    out = pipeline.l1_subspace(A, s=8, r1=16, r2=8, s_out=1e30, seed=1)
    assert out["idx"].size == n
    best = np.inf
    for j in range(d):
        others = [c for c in range(d) if c != j]
        for rows in itertools.combinations(range(n), d - 1):
            M = A[list(rows)][:, others]
            if abs(np.linalg.det(M)) < 1e-12:
                continue
            v = np.linalg.solve(M, A[list(rows), j])
            w = np.zeros(d)
            w[others] = v
            w[j] = -1.0
            best = min(best, np.abs(A @ w).sum())
    assert np.isclose(out["err"][out["j_star"]], best, rtol=1e-9)


def test_subspace_recovers_a_planted_hyperplane():
    rng = np.random.default_rng(4)
    n, d = 4000, 5
    A = rng.standard_normal((n, d))
    normal = np.array([0.5, -1.0, 2.0, 0.25, 1.0])
    A[:, 2] = -(A @ normal - 2.0 * A[:, 2]) / 2.0      # rows on the plane A normal = 0
    A[:, 2] += rng.laplace(0, 1e-3, n)
    A[rng.choice(n, 8, replace=False)] += 5 * rng.standard_cauchy((8, d))
    out = pipeline.l1_subspace(A, s=64, r1=256, r2=16, s_out=800, seed=6)
    w = out["W"][:, out["j_star"]]
    cos = abs(w @ normal) / (np.linalg.norm(w) * np.linalg.norm(normal))
    assert cos > 0.999
    # and the sampled fit is within (1 + eps) of the all-rows one
    full = pipeline.l1_subspace(A, s=64, r1=256, r2=16, s_out=1e30, seed=6)
    assert out["err"][out["j_star"]] <= 1.1 * full["err"][full["j_star"]]
