"""Row-norm estimates, probabilities and the Bernoulli coreset.

FastCauchyRegression figure, steps 4-7:

* Lambda = U Pi2 = X M, lambda_i = median_j |Lambda_ij| (step 5);
* p_i = min{1, s * lambda_i / sum_i lambda_i} (step 6);
* D diagonal, D_ii = 1/p_i with probability p_i and 0 otherwise (step 7);
  the coreset is (D A, D b) restricted to the rows with D_ii != 0.

The figure's caption allows instead exactly s rows drawn independently with
replacement with probabilities p^_i = lambda_i / sum lambda
(``select_with_replacement``); several independent draws from one sampling
pass use instance numbers 0, 1, ... of the random streams.

Readings: the median of an even count is the mean of the two middle order
statistics; the paper's s is the expected coreset size s_out; row i is kept
iff its uniform 32-bit word w_i < T_i = min(2^32, floor(p_i 2^32)), which is
the event "uniform < p_i" on the 2^-32 grid (p_i = 1 keeps the row).  p_i is
formed in FP64 from lambda_i and the FP64 sum.  Definition 'l1 Leverage
Scores' gives the exact quantity lambda estimates, ||U_(i)||_1, used as a
diagnostic.  Test infrastructure only.
"""
from __future__ import annotations

import numpy as np

from . import philox


def row_norm_estimates(X, M) -> np.ndarray:
    """lambda_i = median_j |(X M)_ij| in FP64."""
    lam = np.abs(np.asarray(X, dtype=np.float64) @ np.asarray(M, dtype=np.float64))
    return np.median(lam, axis=1)


def exact_l1_leverage(X, R) -> np.ndarray:
    """||U_(i)||_1 with U = X R^-1 (definition of the l1 leverage scores)."""
    import scipy.linalg
    Ut = scipy.linalg.solve_triangular(np.asarray(R, dtype=np.float64),
                                       np.asarray(X, dtype=np.float64).T, trans="T", lower=False)
    return np.abs(Ut).sum(axis=0)


def probabilities(lam, s_out: float, total=None) -> np.ndarray:
    """p_i = min(1, s_out lambda_i / sum lambda) in FP64."""
    lam = np.asarray(lam, dtype=np.float64)
    if total is None:
        total = float(lam.sum())
    if not total > 0.0:
        return np.ones_like(lam)
    return np.minimum(1.0, float(s_out) * lam / total)


def thresholds(p) -> np.ndarray:
    """T_i = min(2^32, floor(p_i 2^32)) as uint64 (exact: scaling by 2^32 is exact)."""
    t = np.floor(np.asarray(p, dtype=np.float64) * 4294967296.0)
    return np.minimum(t, 4294967296.0).astype(np.uint64)


def select(p, seed: int, instance: int = 0):
    """Indices (ascending) of the kept rows and their weights 1/p_i."""
    p = np.asarray(p, dtype=np.float64)
    words = philox.sample_words(seed, p.shape[0], instance).astype(np.uint64)
    keep = words < thresholds(p)
    idx = np.nonzero(keep)[0]
    return idx, 1.0 / p[idx]


def select_with_replacement(lam, s: int, seed: int, instance: int = 0):
    """Exactly s samples drawn independently with replacement with
    probabilities p^_i = lambda_i / sum lambda (the caption of the
    FastCauchyRegression figure), by inversion: sample j takes the row whose
    interval [C_(i-1), C_i) of the running sums C of lambda contains u_j C_n,
    u_j = (w_j + 1/2) / 2^32 with w_j its stream-4 word.  Returns the rows in
    sample order (repeats included) and the weight 1 / (s p^_i) of each
    sample, so that sum_j weight_j |r_(row_j)| estimates sum_i |r_i|."""
    lam = np.asarray(lam, dtype=np.float64)
    C = np.cumsum(lam)
    total = C[-1]
    u = (philox.replacement_words(seed, s, instance).astype(np.float64) + 0.5) * 2.0 ** -32
    rows = np.searchsorted(C, u * total, side="right")
    rows = np.minimum(rows, lam.shape[0] - 1)
    return rows, total / (s * lam[rows])
