"""GPU parity of the FCT2 transform (section "FCT2 Construction") against the
oracle: Y = Pi1 X element by element within 1e-5 (FP32 data) or 1e-12 (FP64
data) of each output row's l1 scale S_i (the magnitude that bounds the
rounding of any evaluation order), R against the oracle's Gram matrix,
bitwise reproducibility, the (1 + eps) regression that takes its R from
FCT2, and the argument checks.  Shapes cover every block size t from 64 to
4096, s from 1 to 200, ragged n (including n < t), both column-slice widths
and two slices."""
import numpy as np
import pytest
import torch

import synth
from oracle import fct, l1

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


def data(n, d, dtype, seed=0):
    w = synth.scaled(synth.TALL, n, d=d, seed=seed)
    A, b, _ = synth.generate(w)
    return A.astype(dtype), b.astype(dtype)


def xmat(A, b):
    X = A.T.astype(np.float64)
    return X if b is None else np.hstack([X, -b.astype(np.float64)[:, None]])


CASES = [
    # n, d, t, s, r1, dtype, with_b
    (300, 3, 64, 8, 32, np.float32, True),
    (5000, 7, 128, 16, 100, np.float32, True),
    (40000, 16, 1024, 32, 512, np.float32, True),
    (70001, 32, 4096, 64, 1024, np.float32, True),
    (20000, 40, 256, 16, 300, np.float32, False),
    (33333, 9, 2048, 45, 77, np.float32, True),
    (9000, 5, 512, 200, 64, np.float64, True),
    (3000, 2, 2048, 1, 16, np.float64, False),
    (100, 4, 4096, 48, 8, np.float32, True),
    (600000, 5, 1024, 16, 200, np.float32, True),   # 586 blocks: eight overlapped segments
]


@pytest.mark.parametrize("n,d,t,s,r1,dtype,with_b", CASES)
def test_fct2_sketch_parity(F, ctx, n, d, t, s, r1, dtype, with_b):
    print(f"fct2 parity n={n} d={d} t={t} s={s} r1={r1} {np.dtype(dtype).name} b={with_b}", flush=True)
    A, b = data(n, d, dtype, seed=n % 5)
    bb = b if with_b else None
    seed = 777 + n
    Y, _ = F.fct2_sketch(ctx, dev(A), dev(b) if with_b else None, t, s, r1, seed, want_r=False)
    Yg = host(Y).astype(np.float64)
    Yo, S = fct.fct2_apply(xmat(A, bb), t, s, r1, seed, return_scale=True)
    tol = 1e-12 if dtype == np.float64 else 1e-5
    err = np.max(np.abs(Yg - Yo), axis=1)
    print(f"  max err / S = {float(np.max(err / S)):.3e}", flush=True)
    assert np.all(err <= tol * S), float(np.max(err / S))


def test_fct2_r_and_reproducibility(F, ctx):
    n, d, t, s, r1, seed = 120000, 12, 1024, 32, 400, 31
    A, b = data(n, d, np.float32, seed=2)
    Ad, bd = dev(A), dev(b)
    Y1, R1 = F.fct2_sketch(ctx, Ad, bd, t, s, r1, seed)
    Y2, R2 = F.fct2_sketch(ctx, Ad, bd, t, s, r1, seed)
    y1, y2, Rg = host(Y1), host(Y2), host(R1)
    assert np.array_equal(y1, y2) and np.array_equal(Rg, host(R2))
    Yo, S = fct.fct2_apply(xmat(A, b), t, s, r1, seed, return_scale=True)
    assert np.all(np.max(np.abs(y1 - Yo), axis=1) <= 1e-5 * S)
    # R^T R against the oracle's Gram matrix: |d(Y^T Y)_jk| <= 1e-5 sum_i S_i
    # (|Y_ij| + |Y_ik|) + 1e-10 sum_i S_i^2, plus the QR's rounding
    assert np.all(np.diag(Rg) > 0) and np.allclose(np.tril(Rg, -1), 0)
    G = Yo.T @ Yo
    aY = (S[:, None] * np.abs(Yo)).sum(axis=0)
    bound = 1e-5 * (aY[:, None] + aY[None, :]) + 1e-10 * float(S @ S) + 1e-12 * np.abs(G).max()
    assert np.all(np.abs(Rg.T @ Rg - G) <= bound)


def test_fct2_overlap_segments(F, ctx):
    """The launch that runs the contraction of each eighth of the rows on a
    second stream beside the FJLT of the next (a capped, grid-strided FJLT
    grid) against the oracle, run twice (bitwise equal: the partial sums and
    their order are fixed by the plan), and against the one-launch form."""
    A, b = data(1 << 20, 6, np.float32, seed=3)
    Ad, bd = dev(A), dev(b)
    out = {}
    for ov in (1, 0, 1):
        ctx.set_option(F.FCT_OPT_FCT2_OVERLAP, ov)
        Y, R = F.fct2_sketch(ctx, Ad, bd, 1024, 32, 300, 17)
        out.setdefault(ov, []).append((host(Y), host(R)))
    ctx.set_option(F.FCT_OPT_FCT2_OVERLAP, 0)
    (y1, r1), (y3, r3) = out[1]
    (y0, r0), = out[0]
    assert np.array_equal(y1, y3) and np.array_equal(r1, r3)
    Yo, S = fct.fct2_apply(xmat(A, b), 1024, 32, 300, 17, return_scale=True)
    for y in (y0, y1):
        assert np.all(np.max(np.abs(y - Yo), axis=1) <= 1e-5 * S)


def test_fct2_window_of_columns_is_a_column_of_the_whole(F, ctx):
    """Pi1 acts on each column alone: the sketch of one column equals that
    column of the sketch of all (same kernels, bitwise)."""
    A, b = data(50000, 6, np.float32, seed=4)
    Y, _ = F.fct2_sketch(ctx, dev(A), dev(b), 512, 24, 96, 5, want_r=False)
    y = host(Y)
    for j in (0, 3, 5):
        Yj, _ = F.fct2_sketch(ctx, dev(A[j:j + 1]), None, 512, 24, 96, 5, want_r=False)
        assert np.array_equal(host(Yj)[:, 0], y[:, j])


def test_fct2_regression_one_plus_eps(F, ctx):
    w = synth.scaled(synth.TALL, 20000, d=8, seed=6)
    A, b, _ = synth.generate(w)
    eps = 0.05
    prm = F.params(s=1024, r1=256, r2=16, s_out=2000, seed=7, flags=F.FCT_FLAG_FCT2, s2=32)
    x, obj, S = F.l1_regress(ctx, dev(A), dev(b), prm, eps=eps)
    At, bt = A.T.astype(np.float64), b.astype(np.float64)
    _, fopt = l1.lp(At, bt)
    f = l1.objective(At, bt, x)
    print(f"fct2 regression: coreset {S} rows, f / OPT = {f / fopt:.6f}", flush=True)
    assert f <= (1 + eps) * fopt


def test_fct2_argument_checks(F, ctx):
    A, b = data(5000, 4, np.float32)
    Ad, bd = dev(A), dev(b)
    for t, s, r1 in [(96, 8, 64), (32, 8, 64), (8192, 8, 64), (256, 0, 64), (256, 300, 64),
                     (128, 129, 64), (256, 8, 4)]:
        with pytest.raises(F.FctError) as e:
            F.fct2_sketch(ctx, Ad, bd, t, s, r1, 1)
        assert e.value.status == -1, (t, s, r1)
    # FCT2 parameters of the regression: t = s >= 64, 1 <= s2 <= min(t, 256)
    for s, s2 in [(32, 8), (256, 0), (256, 257), (128, 200)]:
        prm = F.params(s=s, r1=64, r2=8, s_out=500, seed=1, flags=F.FCT_FLAG_FCT2, s2=s2)
        with pytest.raises(F.FctError) as e:
            F.l1_regress(ctx, Ad, bd, prm, eps=0.1)
        assert e.value.status == -1, (s, s2)
    # entry points other than l1_regress / l1_coreset reject the flag
    prm = F.params(s=256, r1=64, r2=8, s_out=500, seed=1, flags=F.FCT_FLAG_FCT2, s2=16)
    with pytest.raises(F.FctError) as e:
        F.l1_regress_multi(ctx, Ad, bd, prm, 2)
    assert e.value.status == -1
