"""The whole FastCauchyRegression path (figure l1reg-mainSimp), plainly.

Steps, in the paper's order:

1. X = [A, -b], Pi1 the FCT1 transform;
2. X' = Pi1 X and its QR factorization (R, positive diagonal);
3. Pi2 (q x r2) of independent Cauchys;
4. Lambda = X R^-1 Pi2, computed as X (R^-1 Pi2);
5. lambda_i = median_j |Lambda_ij|;
6. p_i = min{1, s lambda_i / sum lambda};
7. D_ii = 1/p_i with probability p_i;
8. x_hat = argmin ||D A x - D b||_1 by linear programming.

``sampling="replace"`` draws exactly s rows with replacement instead of step
7 (the figure's caption); ``draws`` > 1 takes that many independent draws
(and solves) from the one sampling pass.

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np

from . import basis, fct, l1, lowp, sampling


def form_x(A, b=None) -> np.ndarray:
    A = np.asarray(A, dtype=np.float64)
    if b is None:
        return A
    return np.hstack([A, -np.asarray(b, dtype=np.float64)[:, None]])


def l1_regress(A, b, s: int, r1: int, r2: int, s_out: float, seed: int,
               sign_flip: bool = True, lowp_pass2: bool = False, solve: bool = True,
               pi2: str = "cauchy", sampling_mode: str = "bernoulli", draws: int = 1):
    """Run steps 1-8; return every intermediate in a dict.

    pi2 = "gaussian" runs the optimized regression figure instead: Pi2 of
    independent Gaussians, the same median estimate and the probabilities
    normalized by the sum of the estimates (the figure's p_i = min{1, s
    lambda_i} omits the sum; its proof normalizes, and so does this reading).
    """
    X = form_x(A, b)
    Y = fct.pi1_apply(X, s, r1, seed, sign_flip=sign_flip)
    R = basis.qr_r(Y)
    M = basis.m_matrix(R, seed, r2, pi2=pi2)
    if lowp_pass2:
        Xl = lowp.round_bf16(np.asarray(X, dtype=np.float32))
        Ml = lowp.round_bf16(np.asarray(M, dtype=np.float32))
        lam = sampling.row_norm_estimates(Xl, Ml)
    else:
        lam = sampling.row_norm_estimates(X, M)
    total = float(lam.sum())
    p = sampling.probabilities(lam, s_out, total)
    out = dict(X=X, Y=Y, R=R, M=M, lam=lam, sum_lambda=total, p=p, draws=[])
    A64 = np.asarray(A, dtype=np.float64)
    b64 = None if b is None else np.asarray(b, dtype=np.float64)
    for k in range(draws):
        if sampling_mode == "replace":
            idx, w = sampling.select_with_replacement(lam, int(s_out), seed, k)
        else:
            idx, w = sampling.select(p, seed, k)
        dr = dict(idx=idx, w=w)
        if solve:
            x_hat, f_core = l1.lp(A64[idx], b64[idx], w)
            dr.update(x=x_hat, coreset_objective=f_core, objective=l1.objective(A64, b64, x_hat))
        out["draws"].append(dr)
    out.update(out["draws"][0])
    return out


def l1_regress_mrhs(A, B, s: int, r1: int, r2: int, s_out: float, seed: int,
                    sign_flip: bool = True):
    """Multiple l1 regression (section "Generalizing to Multiple l1
    Regression"): X = [A, -B], the figure's steps 1-7 with q = d + k columns,
    then min_w ||D (A w - B_j)||_1 for every column j of B by LP."""
    A64 = np.asarray(A, dtype=np.float64)
    B64 = np.asarray(B, dtype=np.float64)
    X = np.hstack([A64, -B64])
    Y = fct.pi1_apply(X, s, r1, seed, sign_flip=sign_flip)
    R = basis.qr_r(Y)
    M = basis.m_matrix(R, seed, r2)
    lam = sampling.row_norm_estimates(X, M)
    total = float(lam.sum())
    p = sampling.probabilities(lam, s_out, total)
    idx, w = sampling.select(p, seed)
    k = B64.shape[1]
    W = np.zeros((A64.shape[1], k))
    f = np.zeros(k)
    for j in range(k):
        W[:, j], _ = l1.lp(A64[idx], B64[idx, j], w)
        f[j] = l1.objective(A64, B64[:, j], W[:, j])
    return dict(X=X, R=R, M=M, lam=lam, sum_lambda=total, p=p, idx=idx, w=w, W=W, objective=f)


def l1_subspace(A, s: int, r1: int, r2: int, s_out: float, seed: int, sign_flip: bool = True):
    """l1-norm subspace approximation (section "Application to l1 norm
    Subspace Approximation"): one coreset of X = A (the figure with b empty),
    then for every column j the constrained regression min_{w: w_j = -1}
    ||D A w||_1 by LP, err_j = ||A w_j||_1 on all rows, and j* = argmin."""
    A64 = np.asarray(A, dtype=np.float64)
    n, d = A64.shape
    Y = fct.pi1_apply(A64, s, r1, seed, sign_flip=sign_flip)
    R = basis.qr_r(Y)
    M = basis.m_matrix(R, seed, r2)
    lam = sampling.row_norm_estimates(A64, M)
    total = float(lam.sum())
    p = sampling.probabilities(lam, s_out, total)
    idx, wt = sampling.select(p, seed)
    W = np.zeros((d, d))
    err = np.zeros(d)
    for j in range(d):
        others = [c for c in range(d) if c != j]
        v, _ = l1.lp(A64[idx][:, others], A64[idx, j], wt)
        W[others, j] = v
        W[j, j] = -1.0
        err[j] = float(np.abs(A64 @ W[:, j]).sum())
    return dict(R=R, M=M, lam=lam, sum_lambda=total, p=p, idx=idx, w=wt, W=W, err=err,
                j_star=int(np.argmin(err)))
