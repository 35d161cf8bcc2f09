"""GPU parity of the bucket-owner sketch kernel (FP32, s <= 1024) against the
oracle's Pi1 X, and its bitwise reproducibility.

The kernel is forced through the context option (it is also the default for
r1 <= 1024) and, for r1 > 1024, reached through FCT_FLAG_DETERMINISTIC, which
splits the buckets over several workgroups.  Shapes span one to several
8192-row tiles with ragged tails, r1 that is not a power of two, several
column slices, both sign modes, and windows placed at a global row offset.
The bar is the sketch gate: max_j |Y_ij - Y*_ij| <= 1e-5 S_i, S_i the row's
l1 mass from the oracle.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import fct

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
    c.set_option(F.FCT_OPT_PASS1_KERNEL, F.FCT_P1_OWNER)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _data(n, d, seed=0):
    w = synth.scaled(synth.TALL, n, d=d, seed=seed)
    A, b, _ = synth.generate(w)
    return A.astype(np.float32), b.astype(np.float32)


def _x(A, b):
    X = A.T.astype(np.float64)
    return X if b is None else np.hstack([X, -b.astype(np.float64)[:, None]])


OWNER_CASES = [
    # n, d, s, r1, with_b, sign_flip, row0, deterministic flag
    (1, 1, 2, 2, True, True, 0, False),
    (37, 2, 4, 3, True, True, 0, False),
    (1000, 3, 2, 16, True, True, 0, False),
    (8191, 5, 64, 100, True, False, 0, False),
    (8192, 4, 1024, 1024, True, True, 0, False),
    (20000, 16, 1024, 1024, True, True, 0, False),
    (70001, 7, 128, 513, True, True, 0, False),
    (50000, 20, 512, 600, True, True, 0, False),
    (40000, 33, 256, 512, False, True, 0, False),
    (30000, 3, 8, 256, True, True, 1 << 20, False),
    (25000, 6, 1024, 700, True, False, 3 << 20, False),
    (60000, 12, 256, 2048, True, True, 0, True),
    (30000, 5, 512, 1500, True, True, 0, True),
    (20000, 64, 32, 4096, True, True, 1 << 12, True),
]


@pytest.mark.parametrize("n,d,s,r1,with_b,sign_flip,row0,det", OWNER_CASES)
def test_owner_sketch_parity(F, ctx, n, d, s, r1, with_b, sign_flip, row0, det):
    print(f"owner sketch n={n} d={d} s={s} r1={r1} row0={row0} det={det}", flush=True)
    A, b = _data(n, d, seed=n % 5)
    bb = b if with_b else None
    seed = 99 + n
    flags = (0 if sign_flip else F.FCT_FLAG_NO_SIGN_FLIP) | (F.FCT_FLAG_DETERMINISTIC if det else 0)
    Y = F.fct_sketch_window(ctx, dev(A), dev(bb) if with_b else None, s, r1, seed, row0, flags=flags)
    Yg = host(Y).astype(np.float64)
    Yo, S = fct.pi1_apply(_x(A, bb), s, r1, seed, sign_flip=sign_flip, return_scale=True, row0=row0)
    err = np.max(np.abs(Yg - Yo), axis=1)
    assert np.all(err <= 1e-5 * np.maximum(S, 1e-300)), float(np.max(err / np.maximum(S, 1e-300)))


def test_owner_sketch_bitwise_rerun_and_duplicate_columns(F, ctx):
    A, b = _data(50000, 9, seed=2)
    runs = [host(F.fct_sketch(ctx, dev(A), dev(b), 256, 1024, 5, want_r=False)[0]) for _ in range(3)]
    assert all(np.array_equal(runs[0].view(np.uint32), r.view(np.uint32)) for r in runs[1:])
    Ad = np.vstack([A[:1], A[:1], A[:1]])
    yd = host(F.fct_sketch(ctx, dev(Ad), None, 256, 1024, 5, want_r=False)[0])
    assert np.array_equal(yd[:, 0].view(np.uint32), yd[:, 1].view(np.uint32))
    assert np.array_equal(yd[:, 0].view(np.uint32), yd[:, 2].view(np.uint32))


def test_deterministic_flag_bitwise_at_large_r1(F, ctx):
    A, b = _data(40000, 10, seed=4)
    fl = F.FCT_FLAG_DETERMINISTIC
    runs = [host(F.fct_sketch(ctx, dev(A), dev(b), 512, 3000, 8, flags=fl, want_r=False)[0])
            for _ in range(2)]
    assert np.array_equal(runs[0].view(np.uint32), runs[1].view(np.uint32))


def test_deterministic_flag_rejects_unsupported_shapes(F, ctx):
    A, b = _data(5000, 4, seed=1)
    with pytest.raises(F.FctError) as e:
        F.fct_sketch(ctx, dev(A.astype(np.float64)), dev(b.astype(np.float64)), 64, 256, 1,
                     flags=F.FCT_FLAG_DETERMINISTIC, want_r=False)
    assert e.value.status == -1
    with pytest.raises(F.FctError):
        F.fct_sketch(ctx, dev(A), dev(b), 2048, 256, 1, flags=F.FCT_FLAG_DETERMINISTIC, want_r=False)


def test_owner_and_atomic_kernels_agree_to_tolerance(F, ctx):
    """The same sketch through the owner kernel and the wave kernel with its
    random table: both within the gate of the oracle, hence of each other."""
    A, b = _data(60000, 16, seed=3)
    c2 = F.Context(0)
    try:
        c2.set_option(F.FCT_OPT_PASS1_KERNEL, F.FCT_P1_WAVE)
        Yw = host(F.fct_sketch(c2, dev(A), dev(b), 1024, 1024, 3, want_r=False)[0]).astype(np.float64)
    finally:
        c2.close()
    Yo_ = host(F.fct_sketch(ctx, dev(A), dev(b), 1024, 1024, 3, want_r=False)[0]).astype(np.float64)
    _, S = fct.pi1_apply(_x(A, b), 1024, 1024, 3, return_scale=True)
    assert np.all(np.max(np.abs(Yw - Yo_), axis=1) <= 2e-5 * S)


def test_stream_ordering_without_synchronize(F):
    """A context on torch's default stream: inputs made by torch kernels just
    before the call, temporaries freed right after it and outputs read by torch
    kernels, with no synchronize in between.  The owner sketch is bitwise
    reproducible and doubling X doubles every sum exactly, so each round must
    give exactly twice the reference."""
    c = F.Context(0)
    try:
        n, d = 300000, 16
        A = torch.randn(d, n, device="cuda")
        b = torch.randn(n, device="cuda")
        Y0 = F.fct_sketch(c, A, b, 1024, 1024, 13, want_r=False)[0]
        torch.cuda.synchronize()
        ref = (2.0 * Y0).clone()
        for k in range(4):
            A2, b2 = A * 2.0, b * 2.0          # torch kernels, not waited for
            Y = F.fct_sketch(c, A2, b2, 1024, 1024, 13, want_r=False)[0]
            del A2, b2                          # freed at once
            junk = torch.full((d, n), float(k + 7), device="cuda")  # may reuse their memory
            got = Y * 1.0                       # torch reads the library's output
            del junk
            torch.cuda.synchronize()
            assert torch.equal(got.view(torch.int32), ref.view(torch.int32)), k
    finally:
        c.close()
