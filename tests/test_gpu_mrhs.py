"""Multiple l1 regression and l1 subspace approximation (sections
"Generalizing to Multiple l1 Regression" and "Application to l1 norm Subspace
Approximation") through the C ABI against the oracle.

* l1_regress_mrhs: R against the Gram matrix of the oracle's sketch of
  [A, -B] (the sketch gate carried through), lambda over all rows from the
  GPU's R, the coreset size from the GPU's lambda, and every column's (1 + eps)
  objective (summed by the oracle) against the LP optimum.  With k = 1 the
  path equals l1_regress bit for bit in lambda.
* l1_subspace: the same checks for X = A, every constrained regression's
  objective within (1 + eps) of its LP optimum (n <= 20000; at n = 150000
  within (1 + eps) of the all-rows solve, the certified ratio recorded),
  err_j equal to the oracle's FP64 sum for the GPU's w_j, and j* the argmin.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import basis, fct, l1, philox, sampling

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    from conftest import ensure_built
    ensure_built()
    from paper_1207_4684_amd import fctl1
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return fctl1


@pytest.fixture(scope="module")
def ctx(F):
    c = F.Context(0)
    yield c
    c.close()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def check_r(R, X, s, r1, seed):
    Yo, S = fct.pi1_apply(X, s, r1, seed, return_scale=True)
    assert np.all(np.diag(R) > 0) and np.allclose(np.tril(R, -1), 0)
    G = Yo.T @ Yo
    aY = (S[:, None] * np.abs(Yo)).sum(axis=0)
    bound = 1e-5 * (aY[:, None] + aY[None, :]) + 1e-10 * float(S @ S) + 1e-12 * np.abs(G).max()
    assert np.all(np.abs(R.T @ R - G) <= bound), float(np.max(np.abs(R.T @ R - G) / bound))


def check_lambda_and_count(lam, X, R, seed, r2, s_out, S):
    M = basis.m_matrix(R, seed, r2)
    ref = sampling.row_norm_estimates(X, M)
    scale = (np.abs(X) @ np.abs(M)).max(axis=1)
    assert np.all(np.abs(lam - ref) <= 1e-5 * scale)
    lam64 = lam.astype(np.float64)
    p = sampling.probabilities(lam64, s_out, lam64.sum())
    assert S == int(np.count_nonzero(philox.sample_words(seed, X.shape[0]) < sampling.thresholds(p)))


def design(n, d, k, seed, dtype=np.float32):
    rng = np.random.default_rng(seed)
    A = (rng.standard_normal((n, d)) * 10.0 ** rng.uniform(-1, 1, d)).astype(dtype)
    B = (A.astype(np.float64) @ rng.standard_normal((d, k)) + rng.laplace(0, 0.1, (n, k))).astype(dtype)
    out = rng.choice(n, n // 100, replace=False)
    B[out] = (100 * rng.standard_cauchy((out.size, k))).astype(dtype)
    return A, B


@pytest.mark.parametrize("n,d,k,dtype", [(20000, 6, 3, np.float32), (15001, 4, 5, np.float64),
                                         (200000, 16, 8, np.float32)])
def test_mrhs_against_oracle(F, ctx, n, d, k, dtype):
    A, B = design(n, d, k, n, dtype)
    q = d + k
    s, r1, r2, s_out = 64, 8 * q, 16, 300 * q
    seed = 5 + n
    prm = F.params(s=s, r1=r1, r2=r2, s_out=s_out, seed=seed)
    Ad = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()
    Bd = torch.from_numpy(np.ascontiguousarray(B.T)).cuda()
    Rb = torch.zeros((q, q), dtype=torch.float64, device="cuda")
    lam = torch.zeros(n, dtype=torch.float32, device="cuda")
    W, obj, S, status, st = F.l1_regress_mrhs(ctx, Ad, Bd, prm, R_out=Rb, lambda_out=lam)
    assert st == 0, status
    X = np.hstack([A.astype(np.float64), -B.astype(np.float64)])
    R = host(Rb).T.copy()
    check_r(R, X, s, r1, seed)
    check_lambda_and_count(host(lam), X, R, seed, r2, s_out, S)
    A64 = A.astype(np.float64)
    for j in range(k):
        f = l1.objective(A64, B[:, j].astype(np.float64), W[:, j])
        if n <= 20000:
            fopt = l1.lp(A64, B[:, j].astype(np.float64))[1]
        else:
            x0, _ = F.l1_solve(ctx, Ad, Bd[j], torch.ones(n, dtype=torch.float64, device="cuda"),
                               iters=120)
            fopt = l1.dual_lower_bound(A64, B[:, j].astype(np.float64), x0, stop_at=f / 1.025)
        print(f"mrhs n={n} d={d} k={k} column {j}: S={S} f/opt={f / fopt:.6f}")
        assert f <= 1.05 * fopt, (j, f / fopt)


def test_mrhs_one_column_is_the_simple_regression(F, ctx):
    A, B = design(30000, 8, 1, 3)
    prm = F.params(s=64, r1=128, r2=16, s_out=2000, seed=2)
    Ad = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()
    Bd = torch.from_numpy(np.ascontiguousarray(B.T)).cuda()
    lam = torch.zeros(30000, dtype=torch.float32, device="cuda")
    W, _, S, _, st = F.l1_regress_mrhs(ctx, Ad, Bd, prm, lambda_out=lam)
    assert st == 0
    _, R = F.fct_sketch(ctx, Ad, Bd[0], 64, 128, 2)
    lam1, _, _ = F.l1_sample_probs(ctx, Ad, Bd[0], R, 16, 2, 2000, want_p=False)
    x1, _, S1 = F.l1_regress(ctx, Ad, Bd[0], prm)
    assert np.array_equal(host(lam).view(np.uint32), host(lam1).view(np.uint32))
    assert S == S1


def points(n, d, dtype):
    """Rows near a hyperplane: small n plants one (Laplace noise, a few Cauchy
    outliers); large n takes the regression generator's [A, b] (column
    scales, high-leverage rows, Cauchy outliers in b), whose fits the
    weak-duality certificate bounds tightly."""
    if n <= 20000:
        rng = np.random.default_rng(n)
        A = rng.standard_normal((n, d))
        normal = rng.standard_normal(d)
        A[:, 0] = -(A[:, 1:] @ normal[1:]) / normal[0] + rng.laplace(0, 1e-2, n)
        A[rng.choice(n, n // 200, replace=False)] += 10 * rng.standard_cauchy((n // 200, d))
        return A.astype(dtype)
    w = synth.scaled(synth.TALL, n, d=d - 1)
    Aw, b, _ = synth.generate(w)
    return np.hstack([Aw.T, b[:, None]]).astype(dtype)


@pytest.mark.parametrize("n,d,dtype", [(20000, 5, np.float32), (12000, 3, np.float64),
                                       (150000, 12, np.float32)])
def test_subspace_against_oracle(F, ctx, n, d, dtype):
    A = points(n, d, dtype)
    # the generator's rows for large n: the tall workload's sketch parameters
    s, r1, r2, s_out = (64, 8 * d, 16, 300 * d) if n <= 20000 else (256, 1024, 16, 8000)
    seed = 11 + n
    prm = F.params(s=s, r1=r1, r2=r2, s_out=s_out, seed=seed)
    Ad = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()
    Rb = torch.zeros((d, d), dtype=torch.float64, device="cuda")
    lam = torch.zeros(n, dtype=torch.float32, device="cuda")
    W, err, js, S, status, st = F.l1_subspace(ctx, Ad, prm, R_out=Rb, lambda_out=lam)
    assert st == 0, status
    X = A.astype(np.float64)
    R = host(Rb).T.copy()
    check_r(R, X, s, r1, seed)
    check_lambda_and_count(host(lam), X, R, seed, r2, s_out, S)
    assert np.all(np.diag(W) == -1.0)
    ref_err = np.array([np.abs(X @ W[:, j]).sum() for j in range(d)])
    assert np.allclose(err, ref_err, rtol=1e-10)
    assert js == int(np.argmin(err))
    for j in range(d):
        others = [c for c in range(d) if c != j]
        if n <= 20000:
            # (1 + eps) against the exact LP optimum of regression j
            fopt = l1.lp(X[:, others], X[:, j])[1]
            print(f"subspace n={n} d={d} column {j}: S={S} err/opt={err[j] / fopt:.6f}")
            assert err[j] <= 1.05 * fopt, (j, err[j] / fopt)
        else:
            # large n: no exact optimum; the coreset fit against the all-rows
            # solve of the same regression (f by the oracle), and the
            # weak-duality ratio recorded
            Aj = torch.from_numpy(np.ascontiguousarray(X[:, others].T)).cuda()
            bj = torch.from_numpy(np.ascontiguousarray(X[:, j])).cuda()
            x0, _ = F.l1_solve(ctx, Aj, bj, torch.ones(n, dtype=torch.float64, device="cuda"), iters=120)
            f0 = l1.objective(X[:, others], X[:, j], x0)
            lower = l1.dual_lower_bound(X[:, others], X[:, j], x0, stop_at=err[j] / 1.025)
            print(f"subspace n={n} d={d} column {j}: S={S} err/all-rows={err[j] / f0:.6f} "
                  f"err/certified-lower={err[j] / lower:.6f}")
            assert err[j] <= 1.05 * f0, (j, err[j] / f0)
