"""Well-conditioned basis: R from the QR of the sketch, and M = R^-1 Pi2.

FastL1Basis figure: compute Pi1 A and its QR factorization Pi1 A = Q R; the
basis is U = A R^-1 (never formed here).  FastCauchyRegression figure, steps
2-4: the same with X = [A, -b]; Pi2 in R^{q x r2} is a matrix of independent
Cauchys and Lambda = U Pi2 = X (R^-1 Pi2).  The optimized regression figure
(OptimizedFastCauchyRegression) takes Pi2 Gaussian instead.  The running-time paragraph of the
regression proof computes R^-1 Pi2 first and then X (R^-1 Pi2); so does this
build.

Reading: R is taken with a positive diagonal, which makes it unique for a
full-rank sketch (the paper leaves the signs free; U changes only by column
signs, which leave every |Lambda_ij| distribution and row l1 norm unchanged).
Test infrastructure only.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import philox

RANK_TOL = 1e-13


class RankDeficient(ValueError):
    pass


def qr_r(Y) -> np.ndarray:
    """Upper-triangular R (q x q, positive diagonal) of Y = Q R, in FP64."""
    Y = np.asarray(Y, dtype=np.float64)
    R = np.linalg.qr(Y, mode="r")
    sg = np.where(np.diag(R) < 0, -1.0, 1.0)
    R = sg[:, None] * R
    d = np.abs(np.diag(R))
    if d.size == 0 or not np.all(np.isfinite(R)) or d.min() <= RANK_TOL * d.max():
        raise RankDeficient("sketch is rank deficient")
    return R


def m_matrix(R, seed: int, r2: int, instance: int = 0, pi2: str = "cauchy") -> np.ndarray:
    """M = R^-1 Pi2 (q x r2), by a triangular solve R M = Pi2.

    pi2 = "cauchy": independent Cauchys (FastCauchyRegression figure, step 3);
    pi2 = "gaussian": independent standard Gaussians (the optimized
    regression figure, step 4), whose (U Pi2)_ij are N(0, ||U_(i)||_2^2).
    """
    R = np.asarray(R, dtype=np.float64)
    if pi2 == "cauchy":
        P = philox.pi2_matrix(seed, R.shape[0], r2, instance)
    elif pi2 == "gaussian":
        P = philox.pi2_gaussian_matrix(seed, R.shape[0], r2, instance)
    else:
        raise ValueError(pi2)
    return scipy.linalg.solve_triangular(R, P, lower=False)
