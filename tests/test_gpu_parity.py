"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bars: integer outputs (RNG words, buckets, signs, selected rows, gathered
bytes) bit-exact; Cauchy values within 8 FP32 ulp; Pi1 X within 1e-5 of each
output row's l1 scale; R backward-stable; lambda within 1e-5 of
max_j (|X_i| |M|)_j; the coreset solution's objective within (1 + eps) of the
exact optimum.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import basis, fct, l1, lowp, philox, sampling

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


# ---- random streams --------------------------------------------------------

@pytest.mark.parametrize("stream", [0, 1, 2, 3, 4, 5, 6])
def test_rng_words_bit_exact(F, ctx, stream):
    for idx0 in (0, 2**32 - 5, 2**40 + 3):
        seed = 0x123456789ABCDEF + stream
        got = host(F.fct_rng_words(ctx, stream, seed, idx0, 1000)).view(np.uint32).reshape(-1, 4)
        ref = np.stack(philox.stream_words(seed, stream, np.arange(idx0, idx0 + 1000, dtype=np.uint64)), 1)
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("s", [2, 256, 4096])
def test_pi1_streams_buckets_signs_exact_cauchy_8ulp(F, ctx, s):
    seed, r1 = 77, 2048
    for j0 in (0, 2**33 + 128):
        n = 1 << 16
        bh, ch, bi, ci, sg = (host(t) for t in F.fct_pi1_streams(ctx, seed, r1, s, j0, n))
        j = np.arange(j0, j0 + n, dtype=np.int64)
        kH = 2 * s * (j // s) + j % s
        rbh, rch = philox.position_streams(seed, kH, r1)
        rbi, rci = philox.position_streams(seed, kH + s, r1)
        assert np.array_equal(bh, rbh) and np.array_equal(bi, rbi)
        for got, ref in ((ch, rch), (ci, rci)):
            ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
            assert np.max(np.abs(got.astype(np.float64) - ref) / ulp) <= 8.0
        ncall = (j0 + n + 127) // 128 - j0 // 128
        sw = np.stack(philox.stream_words(seed, 1, np.arange(j0 // 128, j0 // 128 + ncall, dtype=np.uint64)), 1).reshape(-1)
        ju = j.astype(np.uint64)
        word = sw[((ju >> np.uint64(5)) - np.uint64(4 * (j0 // 128))).astype(np.int64)].astype(np.uint64)
        ref_sg = 1 - 2 * ((word >> (ju & np.uint64(31))) & np.uint64(1)).astype(np.int64)
        assert np.array_equal(sg.astype(np.int64), ref_sg)


def test_cauchy_extreme_words(F, ctx):
    # the largest |C| among 2^21 draws (a word near the poles) keeps its sign and value
    bh, ch, bi, ci, sg = (host(t) for t in F.fct_pi1_streams(ctx, 5, 16, 2, 0, 1 << 20))
    _, ref = philox.position_streams(5, np.arange(2 << 20), 16)
    got = np.empty(2 << 20)
    got[0::4], got[1::4] = ch[0::2], ch[1::2]
    got[2::4], got[3::4] = ci[0::2], ci[1::2]
    i = np.argmax(np.abs(ref))
    assert np.sign(got[i]) == np.sign(ref[i]) and abs(got[i] / ref[i] - 1) < 1e-6


# ---- FWHT ------------------------------------------------------------------

@pytest.mark.parametrize("s", [2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096])
def test_fwht_matches_oracle(F, ctx, s):
    nb = max(3, 8192 // s)
    z = np.random.default_rng(s).standard_normal(nb * s).astype(np.float32)
    got = host(F.fct_fwht(ctx, dev(z), s)).reshape(nb, s)
    ref = fct.fwht_blocks(z.astype(np.float64).reshape(nb, s, 1))[:, :, 0]
    tol = 1e-6 * np.linalg.norm(z.reshape(nb, s), axis=1, keepdims=True)
    assert np.all(np.abs(got - ref) <= tol)


# ---- pass 1 ----------------------------------------------------------------

SKETCH_CASES = [
    # n, d, s, r1, dtype, with_b, sign_flip
    (1000, 3, 2, 16, np.float32, True, True),
    (5000, 5, 16, 64, np.float32, False, True),
    (33333, 16, 64, 512, np.float64, True, True),
    (65536, 16, 64, 512, np.float64, True, False),
    (70001, 32, 256, 2048, np.float32, True, True),
    (40000, 7, 1024, 256, np.float32, True, True),
    (20000, 3, 4096, 64, np.float32, True, False),
    (30000, 64, 512, 4096, np.float32, True, True),
    (24000, 5, 2048, 128, np.float32, True, True),
    (10000, 9, 512, 1024, np.float32, True, False),
]


def _data(n, d, dtype, seed=0):
    w = synth.scaled(synth.TALL, n, d=d, seed=seed)
    A, b, _ = synth.generate(w)
    return A.astype(dtype), b.astype(dtype)


@pytest.mark.parametrize("n,d,s,r1,dtype,with_b,sign_flip", SKETCH_CASES)
def test_sketch_parity(F, ctx, n, d, s, r1, dtype, with_b, sign_flip):
    A, b = _data(n, d, dtype, seed=n % 7)
    X = pipeline_x(A, b if with_b else None)
    seed = 1234 + n
    flags = 0 if sign_flip else F.FCT_FLAG_NO_SIGN_FLIP
    Y, R = F.fct_sketch(ctx, dev(A), dev(b) if with_b else None, s, r1, seed, flags=flags,
                        want_r=False)
    Yg = host(Y).astype(np.float64)
    Yo, S = fct.pi1_apply(X, s, r1, seed, sign_flip=sign_flip, return_scale=True)
    err = np.max(np.abs(Yg - Yo), axis=1)
    assert np.all(err <= 1e-5 * S), float(np.max(err / S))


def pipeline_x(A, b):
    X = A.T.astype(np.float64)
    if b is None:
        return X
    return np.hstack([X, -b.astype(np.float64)[:, None]])


def test_sketch_full_size_tall_workload(F, ctx):
    """The benchmark's workload (4,194,304 x 32 FP32, s=256, r1=2048) at full size."""
    w = synth.TALL
    A, b, _ = synth.generate(w)
    Y, _ = F.fct_sketch(ctx, dev(A), dev(b), w.s, w.r1, w.seed, want_r=False)
    Yg = host(Y).astype(np.float64)
    Yo, S = fct.pi1_apply(pipeline_x(A, b), w.s, w.r1, w.seed, return_scale=True)
    err = np.max(np.abs(Yg - Yo), axis=1)
    assert np.all(err <= 1e-5 * S), float(np.max(err / S))


def test_sketch_linearity_and_rerun(F, ctx):
    A, b = _data(20000, 8, np.float32)
    Y1, _ = F.fct_sketch(ctx, dev(A), dev(b), 64, 128, 9, want_r=False)
    Y2, _ = F.fct_sketch(ctx, dev(A), dev(b), 64, 128, 9, want_r=False)
    a1, a2 = host(Y1), host(Y2)
    _, S = fct.pi1_apply(pipeline_x(A, b), 64, 128, 9, return_scale=True)
    assert np.all(np.max(np.abs(a1 - a2), axis=1) <= 1e-6 * S)
    # duplicate columns agree to rounding (LDS atomics add in a run-dependent order)
    Ad = np.vstack([A[:1], A[:1]])
    Yd, _ = F.fct_sketch(ctx, dev(Ad), None, 64, 128, 9, want_r=False)
    yd = host(Yd)
    _, Sd = fct.pi1_apply(Ad.T, 64, 128, 9, return_scale=True)
    assert np.all(np.abs(yd[:, 0] - yd[:, 1]) <= 1e-6 * Sd)


# ---- QR --------------------------------------------------------------------

@pytest.mark.parametrize("n,d,s,r1", [(65536, 16, 64, 512), (50000, 32, 256, 2048), (60000, 64, 512, 4096), (9000, 3, 16, 8)])
def test_qr_parity_fp64(F, ctx, n, d, s, r1):
    A, b = _data(n, d, np.float64, seed=3)
    Y, R = F.fct_sketch(ctx, dev(A), dev(b), s, r1, 5)
    Yg, Rg = host(Y), host(R)
    Ro = basis.qr_r(Yg)
    assert np.allclose(np.tril(Rg, -1), 0) and np.all(np.diag(Rg) > 0)
    scale = np.abs(Ro).max()
    assert np.max(np.abs(Rg - Ro)) <= 1e-10 * scale
    G = Yg.T @ Yg
    assert np.max(np.abs(Rg.T @ Rg - G)) <= 1e-12 * np.abs(G).max()


def test_rank_deficient_reported(F, ctx):
    A, b = _data(4096, 4, np.float32)
    A[2] = A[1]
    with pytest.raises(F.FctError) as e:
        F.fct_sketch(ctx, dev(A), dev(b), 64, 64, 1)
        ctx.sync()
    assert e.value.status == -4


def test_nonfinite_reported(F, ctx):
    A, b = _data(4096, 4, np.float32)
    A[1, 100] = np.nan
    with pytest.raises(F.FctError) as e:
        F.fct_sketch(ctx, dev(A), dev(b), 64, 64, 1, want_r=False)
        ctx.sync()
    assert e.value.status == -3
    ctx.sync()  # flags cleared


# ---- pass 2 ----------------------------------------------------------------

@pytest.mark.parametrize("n,d,s,r1,r2,dtype", [(65536, 16, 64, 512, 8, np.float64),
                                               (1200000, 8, 64, 256, 8, np.float64),  # FP64 grid > 1024 workgroups
                                               (100003, 32, 256, 2048, 16, np.float32),
                                               (70000, 64, 512, 4096, 24, np.float32),
                                               (30000, 5, 64, 64, 3, np.float32),
                                               (30000, 9, 64, 128, 32, np.float32)])
def test_lambda_parity(F, ctx, n, d, s, r1, r2, dtype):
    A, b = _data(n, d, dtype, seed=1)
    seed = 11
    _, R = F.fct_sketch(ctx, dev(A), dev(b), s, r1, seed)
    Rg = host(R)
    lam, p, tot = F.l1_sample_probs(ctx, dev(A), dev(b), R, r2, seed, 1000)
    lam = host(lam).astype(np.float64)
    X = pipeline_x(A, b)
    M = basis.m_matrix(Rg, seed, r2)
    ref = sampling.row_norm_estimates(X, M)
    scale = (np.abs(X) @ np.abs(M)).max(axis=1)
    assert np.all(np.abs(lam - ref) <= 1e-5 * scale + 1e-30)
    assert np.isclose(host(tot)[0], lam.sum(), rtol=1e-12)
    pr = sampling.probabilities(lam, 1000, host(tot)[0])
    assert np.array_equal(host(p), pr.astype(np.float32))


def test_lambda_bf16_parity(F, ctx):
    n, d, s, r1, r2 = 80000, 32, 256, 2048, 16
    A, b = _data(n, d, np.float32, seed=2)
    seed = 21
    _, R = F.fct_sketch(ctx, dev(A), dev(b), s, r1, seed)
    Ab = F.fct_to_bf16(ctx, dev(A))
    bb = F.fct_to_bf16(ctx, dev(b))
    assert np.array_equal(host(Ab).view(np.uint16), lowp.f32_to_bf16_bits(A))
    lam, _, _ = F.l1_sample_probs(ctx, Ab, bb, R, r2, seed, 1000, want_p=False)
    lam = host(lam).astype(np.float64)
    Xl = lowp.round_bf16(pipeline_x(A, b).astype(np.float32))
    Ml = lowp.round_bf16(basis.m_matrix(host(R), seed, r2).astype(np.float32))
    ref = sampling.row_norm_estimates(Xl, Ml)
    scale = (np.abs(Xl) @ np.abs(Ml)).max(axis=1)
    assert np.all(np.abs(lam - ref) <= 1e-5 * scale + 1e-30)


# ---- selection, gather, solve ----------------------------------------------

def test_selection_bit_exact_given_lambda(F, ctx):
    n, d = 200000, 8
    A, b = _data(n, d, np.float32, seed=4)
    _, R = F.fct_sketch(ctx, dev(A), dev(b), 128, 256, 31)
    lam, _, tot = F.l1_sample_probs(ctx, dev(A), dev(b), R, 16, 31, 3000, want_p=False)
    for seed in (31, 32, 2**40 + 1):
        idx, w, S = F.l1_select(ctx, lam, tot, 3000, seed, cap=20000)
        p = sampling.probabilities(host(lam).astype(np.float64), 3000, host(tot)[0])
        oidx, ow = sampling.select(p, seed)
        assert np.array_equal(host(idx), oidx) and np.array_equal(host(w), ow)
        assert abs(S - p.sum()) < 6 * np.sqrt(p.sum())


def test_selection_edge_cases(F, ctx):
    lam = np.zeros(10000, dtype=np.float32)
    lam[[3, 77, 9999]] = 1.0
    tot = np.array([3.0])
    idx, w, S = F.l1_select(ctx, dev(lam), dev(tot), 10**9, 5, cap=100)
    assert list(host(idx)) == [3, 77, 9999] and np.all(host(w) == 1.0)
    with pytest.raises(F.FctError) as e:
        F.l1_select(ctx, dev(np.ones(5000, np.float32)), dev(np.array([5000.0])), 10**9, 5, cap=10)
    assert e.value.status == -6


def test_coreset_gather_exact(F, ctx):
    n, d = 200000, 8
    A, b = _data(n, d, np.float32, seed=4)
    prm = F.params(s=128, r1=256, r2=16, s_out=3000, seed=31)
    At, bt, w, idx, S = F.l1_coreset(ctx, dev(A), dev(b), prm, cap=20000)
    idx = host(idx)
    assert S == idx.size and np.all(np.diff(idx) > 0)
    assert np.array_equal(host(At), A.T[idx]) and np.array_equal(host(bt), b[idx])
    assert np.all(host(w) >= 1.0)


@pytest.mark.parametrize("S,d,dtype", [(500, 1, np.float64), (3000, 5, np.float64), (8000, 32, np.float32), (20000, 64, np.float32)])
def test_weighted_l1_solve(F, ctx, S, d, dtype):
    g = np.random.default_rng(S + d)
    A = (g.standard_normal((S, d)) * 10.0 ** g.uniform(-1, 1, d)).astype(dtype)
    b = (A.astype(np.float64) @ g.standard_normal(d) + g.laplace(size=S) + 50 * g.standard_cauchy(S) * (g.random(S) < 0.05)).astype(dtype)
    w = g.uniform(1.0, 20.0, S)
    x, obj = F.l1_solve(ctx, dev(A.T), dev(b), dev(w))
    _, fopt = l1.lp(A.astype(np.float64), b.astype(np.float64), w)
    f = l1.objective(A.astype(np.float64), b.astype(np.float64), x, w)
    assert f <= fopt * (1 + 1e-6)          # IRLS solver tolerance
    assert np.isclose(obj, f, rtol=1e-9)


def test_regress_all_rows_kept_is_exact(F, ctx):
    """s_out huge: every p_i = 1, the coreset is the whole problem (pin P-10)."""
    A, b = _data(20000, 4, np.float64, seed=5)
    prm = F.params(s=64, r1=64, r2=8, s_out=10**15, seed=1, irls_iters=80)
    x, obj, S = F.l1_regress(ctx, dev(A), dev(b), prm)
    assert S == 20000
    _, fopt = l1.lp(A.T, b)
    assert l1.objective(A.T, b, x) <= fopt * (1 + 1e-7)


def exact_optimum(F, ctx, A64, b64):
    """The optimum (HiGHS LP) for small n, else a certified lower bound on it.

    For large n a candidate comes from the GPU solver on all rows and the
    oracle turns it into a dual-feasible point; weak LP duality makes its value
    a lower bound on the optimum whoever produced the candidate, so
    f(x_hat) <= (1 + eps) * bound implies the (1 + eps) claim."""
    n = A64.shape[0]
    if n <= 20000:  # the LP takes minutes on a box's host cores beyond this
        return l1.lp(A64, b64)[1]
    x0, _ = F.l1_solve(ctx, dev(A64.T), dev(b64), dev(np.ones(n)), iters=120)
    lower = l1.dual_lower_bound(A64, b64, x0)
    assert lower <= l1.objective(A64, b64, x0) * (1 + 1e-12)
    return lower


@pytest.mark.parametrize("name,n,eps", [("small", 65536, 0.05), ("tall", 262144, 0.05)])
def test_regress_one_plus_eps(F, ctx, name, n, eps):
    w = synth.SMALL if name == "small" else synth.scaled(synth.TALL, n)
    A, b, _ = synth.generate(w)
    prm = F.params(s=w.s, r1=w.r1, r2=w.r2, s_out=w.s_out, seed=w.seed)
    x, obj, S = F.l1_regress(ctx, dev(A), dev(b), prm, eps=eps)
    At64, b64 = A.T.astype(np.float64), b.astype(np.float64)
    fopt = exact_optimum(F, ctx, At64, b64)
    f = l1.objective(At64, b64, x)
    print(f"{name}: S={S} ratio={f / fopt:.6f}")
    assert f <= (1 + eps) * fopt, f / fopt
    # the device objective agrees with the host one
    assert np.isclose(F.fct_l1_objective(ctx, dev(A), dev(b), x), f, rtol=1e-9)


def test_argument_checks_with_a_real_context(F, ctx):
    """The argument checks behind the context check: a misaligned window
    start, an empty batch, ldat < S and cap < 1 are FCT_ERR_BAD_ARG with a
    live context and live buffers, and leave the context usable."""
    import ctypes
    lib = F._lib
    h = ctx.handle
    A = torch.zeros((4, 1024), dtype=torch.float32, device="cuda")
    b = torch.zeros(1024, dtype=torch.float32, device="cuda")
    Y = torch.zeros((5, 64), dtype=torch.float32, device="cuda")
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    # row0 not a multiple of s (64), and not of 256
    assert lib.fct_sketch_window(h, P(A), 1024, 4, 1024, F.FCT_F32, P(b), 64, 64, 1, 32, 0, P(Y)) == -1
    assert lib.fct_sketch_window(h, P(A), 1024, 4, 1024, F.FCT_F32, P(b), 64, 64, 1, 128, 0, P(Y)) == -1
    # an empty batch
    inst = (F.fct_instance * 1)()
    x = (ctypes.c_double * 8)()
    status = (ctypes.c_int32 * 1)()
    assert lib.l1_regress_batched(h, inst, 0, F.FCT_F32, 0.05, x, None, None, None, status) == -1
    # ldat < S
    w = torch.ones(1024, dtype=torch.float64, device="cuda")
    assert lib.l1_solve(h, P(A), P(b), P(w), 1024, 4, 512, F.FCT_F32, 0, x, None) == -1
    # cap < 1
    lam = torch.ones(1024, dtype=torch.float32, device="cuda")
    tot = torch.ones(1, dtype=torch.float64, device="cuda")
    idx = torch.zeros(8, dtype=torch.int64, device="cuda")
    S = ctypes.c_int64()
    assert lib.l1_select(h, P(lam), P(tot), 1024, 10, 0, 0, P(idx), P(w), ctypes.byref(S)) == -1
    # the context still works
    Yv, _ = F.fct_sketch(ctx, A, b, 64, 64, 1, want_r=False)
    torch.cuda.synchronize()
    assert torch.count_nonzero(Yv).item() == 0
