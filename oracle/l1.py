"""Exact (weighted) l1 regression optima: the yardstick for every (1+eps) claim.

Problem statement (Introduction, l1 regression): minimize ||A x - b||_1.  Step 8
of the FastCauchyRegression figure solves the coreset problem
min ||D A x - D b||_1 "using linear programming"; with weights w_i = D_ii this
is min sum_i w_i |A_i x - b_i|.

Routes, independent of one another:

* ``lp``           -- the linear program min sum w (u + v) s.t. A x + u - v = b,
                      u, v >= 0, solved by HiGHS;
* ``brute_force``  -- an LP optimum is attained at a vertex, where d rows are
                      interpolated exactly, so the minimum over all d-row
                      subsets B of f(A_B^-1 b_B) is the optimum (tiny n only);
* ``certify_vertex`` -- LP duality: x_B (interpolating the rows B) is optimal
                      iff some y with y_i = w_i sign(r_i) off B and
                      |y_i| <= w_i on B has A^T y = 0;
* ``weighted_median`` / ``separable_optimum`` -- closed form when every row of
                      A is a canonical vector (the paper's large-scale test
                      design): the problem splits per coordinate and each
                      coordinate's optimum is a weighted median.

Test infrastructure only.
"""
from __future__ import annotations

import itertools

import numpy as np


def objective(A, b, x, w=None, chunk: int | None = None) -> float:
    """sum_i w_i |A_i x - b_i| in FP64.  With ``chunk`` the rows are taken
    ``chunk`` at a time (A may then be a large FP32 array or a transposed
    view) and the chunk sums are added in row order."""
    x = np.asarray(x, dtype=np.float64)
    if chunk is None:
        r = np.asarray(A, dtype=np.float64) @ x - np.asarray(b, dtype=np.float64)
        if w is None:
            return float(np.abs(r).sum())
        return float((np.asarray(w, dtype=np.float64) * np.abs(r)).sum())
    total = 0.0
    for lo in range(0, A.shape[0], chunk):
        hi = min(A.shape[0], lo + chunk)
        total += objective(A[lo:hi], b[lo:hi], x, None if w is None else w[lo:hi])
    return total


def brute_force(A, b, w=None):
    """Exact optimum over all d-row interpolating subsets (n <= ~20, d <= 3)."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n, d = A.shape
    best_x, best_f = None, np.inf
    for B in itertools.combinations(range(n), d):
        AB = A[list(B)]
        if abs(np.linalg.det(AB)) < 1e-12 * max(1.0, np.abs(AB).max() ** d):
            continue
        x = np.linalg.solve(AB, b[list(B)])
        f = objective(A, b, x, w)
        if f < best_f:
            best_f, best_x = f, x
    return best_x, best_f


def lp(A, b, w=None):
    """Exact optimum by linear programming (HiGHS)."""
    import scipy.optimize
    import scipy.sparse as sp
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n, d = A.shape
    w = np.ones(n) if w is None else np.asarray(w, dtype=np.float64)
    c = np.concatenate([np.zeros(d), w, w])
    eye = sp.identity(n, format="csr")
    A_eq = sp.hstack([sp.csr_matrix(A), eye, -eye], format="csr")
    bounds = [(None, None)] * d + [(0, None)] * (2 * n)
    res = scipy.optimize.linprog(c, A_eq=A_eq, b_eq=b, bounds=bounds, method="highs")
    if res.status != 0:
        raise RuntimeError(f"LP failed: {res.message}")
    x = res.x[:d]
    return x, objective(A, b, x, w)


def certify_vertex(A, b, x_start, w=None, tol: float = 1e-9):
    """Polish x_start to a vertex and test it with the LP dual.

    Returns (x_vertex, f(x_vertex), optimal, dual_lower_bound).  B is taken as
    the d rows of smallest |residual| that are linearly independent.  The
    dual y is scaled into the box if needed, giving the lower bound
    b^T y / ... = sum y_i b_i (valid for any feasible dual).
    """
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n, d = A.shape
    w = np.ones(n) if w is None else np.asarray(w, dtype=np.float64)
    r = A @ np.asarray(x_start, dtype=np.float64) - b
    order = np.argsort(np.abs(r), kind="stable")
    B = []
    for i in order:
        cand = B + [int(i)]
        if np.linalg.matrix_rank(A[cand], tol=1e-10 * max(1.0, np.abs(A[cand]).max())) == len(cand):
            B = cand
        if len(B) == d:
            break
    if len(B) < d:
        return np.asarray(x_start, dtype=np.float64), objective(A, b, x_start, w), False, -np.inf
    AB = A[B]
    xv = np.linalg.solve(AB, b[B])
    r = A @ xv - b
    inB = np.zeros(n, dtype=bool)
    inB[B] = True
    y = np.where(inB, 0.0, w * np.sign(r))
    rhs = -(A[~inB].T @ y[~inB])
    yB = np.linalg.solve(AB.T, rhs)
    y[B] = yB
    ratio = np.max(np.abs(yB) / w[B]) if d else 0.0
    optimal = bool(ratio <= 1.0 + tol)
    # A^T y = 0 holds by construction; scale into the box |y_i| <= w_i.
    ys = y / max(1.0, ratio)
    # weak duality: for A^T y = 0 and |y_i| <= w_i, sum w|r| >= -sum y_i b_i
    lower = float(-(ys @ b))
    return xv, objective(A, b, xv, w), optimal, lower


def dual_lower_bound(A, b, x, w=None, rank_taus_only: bool = False, chunk: int = 1 << 20,
                     threads: int = 1, max_free: int | None = None, stop_at: float | None = None):
    """A certified lower bound on min_x sum_i w_i |A_i x - b_i| (weak LP duality).

    For any y with A^T y = 0 and |y_i| <= w_i, and any x,
    sum_i w_i |r_i(x)| >= sum_i y_i r_i(x) = -y^T b.  y is built from a
    candidate x: y_i = w_i clip(r_i / tau, -1, 1) (the subgradient of the
    l1 term, smoothed on |r| <= tau); the violation A^T y is removed by the
    minimum-norm correction supported on the free rows F = {|r_i| < tau}
    (rows whose y_i is inside the box), and y is finally scaled into the box.
    At a vertex with tau between the d interpolated residuals and the rest,
    F is the basis and this is the classical certificate.  Several tau are
    tried; the best bound is returned.  Valid whatever produced x (up to the
    rounding of A^T y = 0); tight when x is optimal.

    Products with A are formed in FP64 over row chunks (optionally on several
    threads), so A may be a large FP32 array.  ``rank_taus_only`` tries only
    the tau placed just above the d-th, (d+1)-th, 2d-th and 4d-th smallest
    |r_i| (small free sets; enough when x is exactly at a vertex).
    ``max_free`` skips tau whose free set has more rows; ``stop_at`` ends the
    search once a bound reaches it, trying first the tau nearest (in ratio)
    to the one just above the d smallest residuals.
    """
    from concurrent.futures import ThreadPoolExecutor

    b = np.asarray(b, dtype=np.float64)
    n, d = A.shape
    w = np.ones(n) if w is None else np.asarray(w, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    starts = list(range(0, n, chunk))

    def rows(lo):
        return np.asarray(A[lo:min(n, lo + chunk)], dtype=np.float64)

    def pmap(fn):
        if threads > 1 and len(starts) > 1:
            with ThreadPoolExecutor(max_workers=threads) as ex:
                return list(ex.map(fn, starts))
        return [fn(lo) for lo in starts]

    def pmap_list(items, fn):
        if threads > 1 and len(items) > 1:
            with ThreadPoolExecutor(max_workers=threads) as ex:
                return list(ex.map(fn, items))
        return [fn(it) for it in items]

    def matvec(v):
        return np.concatenate(pmap(lambda lo: rows(lo) @ v))

    def rmatvec(y, absolute=False):
        if absolute:
            parts = pmap(lambda lo: np.abs(rows(lo)).T @ np.abs(y[lo:lo + chunk]))
        else:
            parts = pmap(lambda lo: rows(lo).T @ y[lo:lo + chunk])
        return np.sum(parts, axis=0)

    r = matvec(x) - b
    absr = np.abs(r)
    ks = sorted({min(n - 1, k) for k in (d - 1, d, 2 * d, 4 * d)})
    part = np.partition(absr, ks)
    ranks = [part[k] * 1.0001 for k in ks]
    scale_r = float(absr.max()) or 1.0
    if rank_taus_only:
        taus = sorted(set(ranks))
    else:
        taus = sorted(set(np.concatenate([scale_r * 10.0 ** np.arange(-16.0, 0.5, 0.5), ranks])))
    if stop_at is not None:
        ref = max(ranks[min(1, len(ranks) - 1)], 1e-300)
        taus = sorted(taus, key=lambda t: abs(np.log(max(t, 1e-300) / ref)))
    absAw = rmatvec(w, absolute=True).max()   # |A|^T |y| <= |A|^T w for |y| <= w
    best = -np.inf
    for tau in taus:
        if not tau > 0:
            continue
        y = w * np.clip(r / tau, -1.0, 1.0)
        free = absr < tau
        nf = int(free.sum())
        if nf < d or (rank_taus_only and nf > 64 * d) or (max_free is not None and nf > max_free):
            continue
        fidx = np.flatnonzero(free)
        g = rmatvec(y)
        if nf <= (1 << 16):
            AF = np.asarray(A[fidx], dtype=np.float64)
            delta, *_ = np.linalg.lstsq(AF.T, -g, rcond=None)
            res = g + AF.T @ delta
        else:
            # minimum-norm correction delta = A_F z with (A_F^T A_F) z = -g,
            # solved after equilibrating the columns; formed over row chunks
            fch = [fidx[i:i + chunk] for i in range(0, nf, chunk)]
            K = np.sum(pmap_list(fch, lambda ix: (lambda B: B.T @ B)(np.asarray(A[ix], dtype=np.float64))),
                       axis=0)
            sc_c = 1.0 / np.sqrt(np.maximum(np.diag(K), 1e-300))
            z = sc_c * np.linalg.solve(K * np.outer(sc_c, sc_c), -g * sc_c)
            delta = np.concatenate(pmap_list(fch, lambda ix: np.asarray(A[ix], dtype=np.float64) @ z))
            res = g + np.sum(pmap_list([np.arange(i, min(nf, i + chunk)) for i in range(0, nf, chunk)],
                                       lambda ii: np.asarray(A[fidx[ii]], dtype=np.float64).T @ delta[ii]),
                             axis=0)
        y[fidx] += delta
        sc = max(1.0, float(np.max(np.abs(y) / w)))
        # A^T y after the correction is g + A_F^T delta (no further pass over A)
        if np.linalg.norm(res) > 1e-9 * absAw * sc:
            continue
        best = max(best, float(-(y / sc) @ b))
        if stop_at is not None and best >= stop_at:
            break
    return best


def weighted_median(values, weights=None) -> float:
    """A minimizer of sum_i w_i |x - v_i| (lower weighted median)."""
    v = np.asarray(values, dtype=np.float64)
    wt = np.ones_like(v) if weights is None else np.asarray(weights, dtype=np.float64)
    order = np.argsort(v, kind="stable")
    cw = np.cumsum(wt[order])
    k = int(np.searchsorted(cw, 0.5 * cw[-1]))
    return float(v[order][k])


def separable_optimum(coord, b, d: int, w=None) -> np.ndarray:
    """Optimum when row i of A is the canonical vector e_{coord[i]}."""
    coord = np.asarray(coord)
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros(d)
    for c in range(d):
        sel = coord == c
        x[c] = weighted_median(b[sel], None if w is None else np.asarray(w)[sel])
    return x
