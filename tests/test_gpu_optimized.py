"""GPU parity of the optimized regression (OptimizedFastCauchyRegression
figure): Gaussian Pi2 through FCT_FLAG_GAUSSIAN_PI2.

* lambda with Gaussian Pi2 against the oracle (FP32 and BF16 streams), with
  the pass-2 bar of the plain method (1e-5 of max_j (|X_i| |M|)_j);
* the probabilities bit-exact given lambda and the sum, normalized (reading of
  the figure's p_i = min{1, s lambda_i});
* the whole optimized path: f(x_hat) <= (1 + eps) f(x_opt), with the exact LP
  optimum (small) or a weak-duality lower bound from the oracle (tall).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import basis, l1, lowp, sampling

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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _x(A, b):
    return np.hstack([A.T.astype(np.float64), -b.astype(np.float64)[:, None]])


@pytest.mark.parametrize("n,d,s,r1,r2,dtype", [(65536, 16, 64, 512, 6, np.float64),
                                               (100003, 32, 256, 2048, 8, np.float32),
                                               (50000, 16, 1024, 1024, 8, np.float32),
                                               (30000, 5, 64, 64, 3, np.float32)])
def test_gaussian_lambda_parity(F, ctx, n, d, s, r1, r2, dtype):
    w = synth.scaled(synth.TALL, n, d=d, seed=1)
    A, b, _ = synth.generate(w)
    A, b = A.astype(dtype), b.astype(dtype)
    seed = 17
    _, R = F.fct_sketch(ctx, dev(A), dev(b), s, r1, seed)
    lam, p, tot = F.l1_sample_probs(ctx, dev(A), dev(b), R, r2, seed, 1000,
                                    flags=F.FCT_FLAG_GAUSSIAN_PI2)
    lam = host(lam).astype(np.float64)
    X = _x(A, b)
    M = basis.m_matrix(host(R), seed, r2, pi2="gaussian")
    ref = sampling.row_norm_estimates(X, M)
    scale = (np.abs(X) @ np.abs(M)).max(axis=1)
    assert np.all(np.abs(lam - ref) <= 1e-5 * scale + 1e-30)
    pr = sampling.probabilities(lam, 1000, host(tot)[0])
    assert np.array_equal(host(p), pr.astype(np.float32))
    assert pr.sum() <= 1000 * (1 + 1e-9)


def test_gaussian_lambda_bf16_parity(F, ctx):
    w = synth.scaled(synth.TALL, 80000, d=32, seed=2)
    A, b, _ = synth.generate(w)
    seed = 23
    _, R = F.fct_sketch(ctx, dev(A), dev(b), 256, 2048, seed)
    Ab, bb = F.fct_to_bf16(ctx, dev(A)), F.fct_to_bf16(ctx, dev(b))
    lam, _, _ = F.l1_sample_probs(ctx, Ab, bb, R, 8, seed, 1000, want_p=False,
                                  flags=F.FCT_FLAG_GAUSSIAN_PI2)
    lam = host(lam).astype(np.float64)
    Xl = lowp.round_bf16(_x(A, b).astype(np.float32))
    Ml = lowp.round_bf16(basis.m_matrix(host(R), seed, 8, pi2="gaussian").astype(np.float32))
    ref = sampling.row_norm_estimates(Xl, Ml)
    scale = (np.abs(Xl) @ np.abs(Ml)).max(axis=1)
    assert np.all(np.abs(lam - ref) <= 1e-5 * scale + 1e-30)


@pytest.mark.parametrize("name,n,r2,eps", [("small", 65536, 6, 0.05), ("tall", 262144, 8, 0.05)])
def test_optimized_regress_one_plus_eps(F, ctx, name, n, r2, eps):
    w = synth.SMALL if name == "small" else synth.scaled(synth.TALL, n)
    A, b, _ = synth.generate(w)
    prm = F.params(s=w.s, r1=w.r1, r2=r2, s_out=w.s_out, seed=w.seed,
                   flags=F.FCT_FLAG_GAUSSIAN_PI2)
    x, obj, S = F.l1_regress(ctx, dev(A), dev(b), prm, eps=eps)
    At64, b64 = A.T.astype(np.float64), b.astype(np.float64)
    if n <= 20000:
        fopt = l1.lp(At64, b64)[1]
    else:
        x0, _ = F.l1_solve(ctx, dev(At64.T), dev(b64), dev(np.ones(n)), iters=120)
        fopt = l1.dual_lower_bound(At64, b64, x0)
    f = l1.objective(At64, b64, x)
    print(f"optimized {name}: S={S} ratio={f / fopt:.6f}")
    assert f <= (1 + eps) * fopt, f / fopt
