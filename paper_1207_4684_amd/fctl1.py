"""Python binding of libfctl1.so: argument marshalling only.

Every computation runs in the HIP library (include/fctl1.h); this module
turns torch device tensors into pointers and sizes, calls the C entry point
of the same name and raises on a non-zero status.  Matrices use the
library's column-major convention: an n x d matrix A is stored as a torch
tensor of shape (d, n) (row j is column j).  There is no CPU fallback: the
module raises ImportError when the built library is absent.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loaded first so the library binds to the same HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfctl1.so")

FCT_F32, FCT_F64, FCT_BF16 = 0, 1, 2
FCT_SAMPLE_BERNOULLI, FCT_SAMPLE_REPLACE = 0, 1
FCT_FLAG_NO_SIGN_FLIP = 1
FCT_FLAG_DETERMINISTIC = 2
FCT_FLAG_GAUSSIAN_PI2 = 4
FCT_FLAG_FCT2 = 8
FCT_OPT_PASS1_KERNEL, FCT_OPT_PASS1_WGS_PER_CU, FCT_OPT_PASS1_TILE_THREADS = 1, 2, 3
FCT_OPT_PASS2_WGS, FCT_OPT_SOLVE_WGS, FCT_OPT_SOLVE_ROWS, FCT_OPT_FCT2_OVERLAP = 4, 5, 6, 7
FCT_P1_AUTO, FCT_P1_WAVE, FCT_P1_OWNER, FCT_P1_TILE = 0, 1, 2, 3
STATUS = {0: "ok", -1: "bad argument", -2: "out of device memory", -3: "non-finite value in input",
          -4: "rank deficient", -5: "HIP runtime error", -6: "coreset larger than capacity"}


class FctError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {STATUS.get(status, status)} ({status})")
        self.status = status


class fct_params(ctypes.Structure):
    _fields_ = [("s", ctypes.c_int32), ("r1", ctypes.c_int32), ("r2", ctypes.c_int32),
                ("s2", ctypes.c_int32), ("s_out", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("flags", ctypes.c_uint32), ("irls_iters", ctypes.c_int32)]


class fct_instance(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("b", ctypes.c_void_p), ("A_lowp", ctypes.c_void_p),
                ("b_lowp", ctypes.c_void_p), ("n", ctypes.c_int64), ("lda", ctypes.c_int64),
                ("ld_lowp", ctypes.c_int64), ("d", ctypes.c_int32), ("pad0", ctypes.c_int32),
                ("prm", fct_params), ("R_out", ctypes.c_void_p), ("lambda_out", ctypes.c_void_p),
                ("idx_out", ctypes.c_void_p), ("idx_cap", ctypes.c_int64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                          "python paper_1207_4684_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U32, U64, D = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                ctypes.c_uint64, ctypes.c_double)
    PD, PI64 = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)
    sig = {
        "fct_create": (ctypes.c_int, [ctypes.POINTER(P), ctypes.c_int, P]),
        "fct_destroy": (None, [P]),
        "fct_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "fct_sync": (ctypes.c_int, [P]),
        "fct_stream": (P, [P]),
        "fct_sketch": (ctypes.c_int, [P, P, I64, I32, I64, ctypes.c_int, P, I32, I32, U64, U32, P, P]),
        "fct_sketch_window": (ctypes.c_int, [P, P, I64, I32, I64, ctypes.c_int, P, I32, I32, U64,
                                             I64, U32, P]),
        "fct2_sketch": (ctypes.c_int, [P, P, I64, I32, I64, ctypes.c_int, P, I32, I32, I32, U64, P, P]),
        "l1_sample_probs": (ctypes.c_int, [P, P, P, I64, I32, I64, ctypes.c_int, P, I32, U64, I64,
                                           P, P, P]),
        "l1_sample_probs_ex": (ctypes.c_int, [P, P, P, I64, I32, I64, ctypes.c_int, P, I32, U64,
                                              I64, U32, P, P, P]),
        "l1_sample_probs_noalloc": (ctypes.c_int, [P, P, P, I64, I32, I64, ctypes.c_int, P, I32,
                                                   U64, I64, U32, P, P, P]),
        "l1_coreset": (ctypes.c_int, [P, P, P, I64, I32, I64, ctypes.c_int, P, P, I64,
                                      ctypes.POINTER(fct_params), I64, P, P, P, P, PI64]),
        "l1_regress": (ctypes.c_int, [P, P, P, I64, I32, I64, ctypes.c_int, P, P, I64, D,
                                      ctypes.POINTER(fct_params), PD, PD, PI64]),
        "fct_rng_words": (ctypes.c_int, [P, U32, U64, U64, I64, P]),
        "fct_pi1_streams": (ctypes.c_int, [P, U64, I32, I32, U64, I64, P, P, P, P, P]),
        "fct_fwht": (ctypes.c_int, [P, P, I64, I32]),
        "fct_to_bf16": (ctypes.c_int, [P, P, I64, P]),
        "fct_lowp_residual": (ctypes.c_int, [P, P, P, I64, I32, I64, ctypes.c_int, P, P, P]),
        "l1_select_draw": (ctypes.c_int, [P, P, P, I64, I64, U64, I32, I32, I64, P, P, PI64]),
        "l1_regress_mrhs": (ctypes.c_int, [P, P, P, I64, I32, I32, I64, I64, ctypes.c_int, D,
                                           ctypes.POINTER(fct_params), PD, PD, PI64,
                                           ctypes.POINTER(ctypes.c_int32), P, P]),
        "l1_subspace": (ctypes.c_int, [P, P, I64, I32, I64, ctypes.c_int, D,
                                       ctypes.POINTER(fct_params), PD, PD,
                                       ctypes.POINTER(ctypes.c_int32), PI64,
                                       ctypes.POINTER(ctypes.c_int32), P, P]),
        "fct_l1_objectives": (ctypes.c_int, [P, P, P, I64, I32, I32, I64, I64, ctypes.c_int, PD, PD]),
        "l1_regress_multi": (ctypes.c_int, [P, P, P, I64, I32, I64, ctypes.c_int, D,
                                            ctypes.POINTER(fct_params), I32, I32, PD, PD, PI64,
                                            ctypes.POINTER(ctypes.c_int32)]),
        "fct_l1_objective": (ctypes.c_int, [P, P, P, I64, I32, I64, ctypes.c_int, PD, PD]),
        "l1_solve": (ctypes.c_int, [P, P, P, P, I64, I32, I64, ctypes.c_int, I32, PD, PD]),
        "l1_select": (ctypes.c_int, [P, P, P, I64, I64, U64, I64, P, P, PI64]),
        "l1_regress_batched": (ctypes.c_int, [P, ctypes.POINTER(fct_instance), I32, ctypes.c_int, D,
                                              PD, PD, PI64, ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(ctypes.c_int32)]),
        "fct_profile": (ctypes.c_int, [P, ctypes.c_int]),
        "fct_set_option": (ctypes.c_int, [P, ctypes.c_int, I64]),
        "fct_profile_read": (ctypes.c_int, [P, ctypes.c_int, PD, PI64]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()
EXPORTED = ("fct_create", "fct_destroy", "fct_strerror", "fct_sync", "fct_stream", "fct_sketch",
            "fct_sketch_window", "l1_sample_probs", "l1_sample_probs_ex", "l1_sample_probs_noalloc",
            "l1_coreset", "l1_regress", "fct_rng_words", "fct_pi1_streams", "fct_fwht",
            "fct_to_bf16", "fct_lowp_residual", "fct_l1_objective", "l1_solve", "l1_select",
            "fct_profile", "fct_profile_read", "l1_regress_batched", "fct_set_option",
            "l1_select_draw", "l1_regress_multi", "l1_regress_mrhs", "l1_subspace",
            "fct_l1_objectives", "fct2_sketch")


def _check(st: int, where: str):
    if st != 0:
        raise FctError(st, where)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    return ctypes.c_void_p(t.data_ptr())


def _dt(t):
    if t.dtype == torch.float32:
        return FCT_F32
    if t.dtype == torch.float64:
        return FCT_F64
    if t.dtype in (torch.bfloat16, torch.int16, torch.uint16):
        return FCT_BF16
    raise TypeError(f"unsupported dtype {t.dtype}")


def _cm(A):
    """(d, n) row-major storage of a column-major n x d matrix: returns n, d, lda."""
    if A.dim() != 2 or (A.stride(1) != 1 and A.shape[1] > 1):
        raise ValueError("A must be a (d, n) tensor with unit stride along n")
    # a leading dimension of size 1 may carry any stride
    return A.shape[1], A.shape[0], (A.stride(0) if A.shape[0] > 1 else A.shape[1])


class Context:
    """fct_create / fct_destroy on a device.

    The library enqueues on its context's stream.  When torch's current stream
    is the legacy default stream (handle 0) the library creates a stream of
    its own, which is not ordered with torch's; every call through this
    module is therefore bracketed: the library's stream first waits for
    torch's current stream (inputs written by torch are complete), and torch's
    current stream then waits for the library's (its outputs are complete
    before torch reads them or reuses the memory of temporaries freed after
    the call).  With a stream of the caller's choosing the two coincide and
    the bracket is empty."""

    def __init__(self, device: int = 0, stream=None):
        dev = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        self.device = device
        h = ctypes.c_void_p()
        _check(_lib.fct_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream)),
               "fct_create")
        self.handle = h
        self.lib_stream = _lib.fct_stream(h) or 0
        self.stream = (stream if self.lib_stream == stream.cuda_stream
                       else torch.cuda.ExternalStream(self.lib_stream, device=dev))

    def call(self, fn, *args):
        """fn(*args) with the library's stream ordered after torch's current
        stream, and torch's current stream ordered after the library's."""
        cur = torch.cuda.current_stream(self.device)
        same = cur.cuda_stream == self.lib_stream
        if not same:
            self.stream.wait_stream(cur)
        st = fn(*args)
        if not same:
            cur.wait_stream(self.stream)
        return st

    def close(self):
        if self.handle:
            _lib.fct_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self):
        _check(self.call(_lib.fct_sync, self.handle), "fct_sync")

    def set_option(self, option: int, value: int):
        """fct_set_option: plan options (pass-1 kernel, grid sizes)."""
        _check(_lib.fct_set_option(self.handle, option, int(value)), "fct_set_option")

    def profile(self, enable: bool):
        _check(_lib.fct_profile(self.handle, 1 if enable else 0), "fct_profile")

    def profile_read(self, kind: int):
        """(total device ms, launches) of kind 0 = pass 1, 1 = pass 2, 2 = solve."""
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        _check(_lib.fct_profile_read(self.handle, kind, ctypes.byref(ms), ctypes.byref(cnt)),
               "fct_profile_read")
        return ms.value, cnt.value


def params(s, r1, r2, s_out, seed, flags=0, irls_iters=0, s2=0):
    """fct_params; with FCT_FLAG_FCT2, s is FCT2's block size t and s2 its s."""
    return fct_params(s=s, r1=r1, r2=r2, s2=s2, s_out=int(s_out), seed=seed, flags=flags,
                      irls_iters=irls_iters)


def fct_sketch(ctx, A, b, s, r1, seed, flags=0, want_y=True, want_r=True):
    """Y = Pi1 X (r1 x q view) and R (q x q view, FP64) of its QR."""
    n, d, lda = _cm(A)
    q = d + (1 if b is not None else 0)
    Y = torch.empty((q, r1), dtype=A.dtype, device=A.device) if want_y else None
    R = torch.empty((q, q), dtype=torch.float64, device=A.device) if want_r else None
    _check(ctx.call(_lib.fct_sketch, ctx.handle, _ptr(A), n, d, lda, _dt(A), _ptr(b), s, r1, seed, flags,
                           _ptr(Y), _ptr(R)), "fct_sketch")
    return (Y.t() if Y is not None else None), (R.t() if R is not None else None)


def fct2_sketch(ctx, A, b, t, s, r1, seed, want_y=True, want_r=True):
    """Y = Pi1 X with FCT2 (r1 x q view) and R (q x q view, FP64)."""
    n, d, lda = _cm(A)
    q = d + (1 if b is not None else 0)
    Y = torch.empty((q, r1), dtype=A.dtype, device=A.device) if want_y else None
    R = torch.empty((q, q), dtype=torch.float64, device=A.device) if want_r else None
    _check(ctx.call(_lib.fct2_sketch, ctx.handle, _ptr(A), n, d, lda, _dt(A), _ptr(b), t, s, r1, seed,
                    _ptr(Y), _ptr(R)), "fct2_sketch")
    return (Y.t() if Y is not None else None), (R.t() if R is not None else None)


def fct_sketch_window(ctx, A, b, s, r1, seed, row0, flags=0):
    """The share of Pi1 X from a window of rows starting at global row ``row0``
    (A, b are the window's rows); returns the r1 x q view."""
    n, d, lda = _cm(A)
    q = d + (1 if b is not None else 0)
    Y = torch.empty((q, r1), dtype=A.dtype, device=A.device)
    _check(ctx.call(_lib.fct_sketch_window, ctx.handle, _ptr(A), n, d, lda, _dt(A), _ptr(b), s, r1, seed,
                                  int(row0), flags, _ptr(Y)), "fct_sketch_window")
    return Y.t()


def l1_sample_probs(ctx, A, b, R, r2, seed, s_out, want_p=True, flags=0):
    """lambda (n, FP32), p (n, FP32) and sum lambda (FP64 device scalar).
    flags = FCT_FLAG_GAUSSIAN_PI2 calls l1_sample_probs_ex (Gaussian Pi2)."""
    n, d, lda = _cm(A)
    Rbuf = R.t().contiguous()  # column-major q x q storage of the logical R
    lam = torch.empty(n, dtype=torch.float32, device=A.device)
    p = torch.empty(n, dtype=torch.float32, device=A.device) if want_p else None
    tot = torch.empty(1, dtype=torch.float64, device=A.device)
    if flags:
        _check(ctx.call(_lib.l1_sample_probs_ex, ctx.handle, _ptr(A), _ptr(b), n, d, lda, _dt(A), _ptr(Rbuf),
                                       r2, seed, int(s_out), flags, _ptr(lam), _ptr(p), _ptr(tot)),
               "l1_sample_probs_ex")
    else:
        _check(ctx.call(_lib.l1_sample_probs, ctx.handle, _ptr(A), _ptr(b), n, d, lda, _dt(A), _ptr(Rbuf),
                                    r2, seed, int(s_out), _ptr(lam), _ptr(p), _ptr(tot)),
               "l1_sample_probs")
    return lam, p, tot


def l1_sample_probs_noalloc(ctx, A, b, R, r2, seed, s_out, lam, tot, p=None, flags=0):
    """l1_sample_probs_noalloc: lambda, p, sum lambda into caller-provided
    device tensors (lam FP32 [n], tot FP64 [1], p FP32 [n] or None)."""
    n, d, lda = _cm(A)
    Rbuf = R.t().contiguous()
    _check(ctx.call(_lib.l1_sample_probs_noalloc, ctx.handle, _ptr(A), _ptr(b), n, d, lda, _dt(A), _ptr(Rbuf),
                                        r2, seed, int(s_out), flags, _ptr(lam), _ptr(p), _ptr(tot)),
           "l1_sample_probs_noalloc")
    return lam, p, tot


def l1_coreset(ctx, A, b, prm, cap, A_lowp=None, b_lowp=None):
    """(At (S x d view), bt, w, idx, S) of the Bernoulli coreset."""
    n, d, lda = _cm(A)
    At = torch.empty((d, cap), dtype=A.dtype, device=A.device)
    bt = torch.empty(cap, dtype=A.dtype, device=A.device)
    w = torch.empty(cap, dtype=torch.float64, device=A.device)
    idx = torch.empty(cap, dtype=torch.int64, device=A.device)
    S = ctypes.c_int64()
    ld_lowp = A_lowp.stride(0) if A_lowp is not None else 0
    st = ctx.call(_lib.l1_coreset, ctx.handle, _ptr(A), _ptr(b), n, d, lda, _dt(A), _ptr(A_lowp),
                         _ptr(b_lowp), ld_lowp, ctypes.byref(prm), cap, _ptr(At), _ptr(bt),
                         _ptr(w), _ptr(idx), ctypes.byref(S))
    _check(st, "l1_coreset")
    k = S.value
    return At[:, :k].t(), bt[:k], w[:k], idx[:k], k


def l1_regress(ctx, A, b, prm, eps=0.05, A_lowp=None, b_lowp=None):
    """x (numpy FP64), coreset objective, realised coreset size."""
    import numpy as np
    n, d, lda = _cm(A)
    x = (ctypes.c_double * d)()
    obj = ctypes.c_double()
    S = ctypes.c_int64()
    ld_lowp = A_lowp.stride(0) if A_lowp is not None else 0
    st = ctx.call(_lib.l1_regress, ctx.handle, _ptr(A), _ptr(b), n, d, lda, _dt(A), _ptr(A_lowp),
                         _ptr(b_lowp), ld_lowp, eps, ctypes.byref(prm), x, ctypes.byref(obj),
                         ctypes.byref(S))
    _check(st, "l1_regress")
    return np.array(x[:], dtype=np.float64), obj.value, S.value


def l1_select(ctx, lam, sum_lambda, s_out, seed, cap):
    """idx (ascending), w = 1/p and S of one Bernoulli draw from given lambda."""
    n = lam.numel()
    idx = torch.empty(cap, dtype=torch.int64, device=lam.device)
    w = torch.empty(cap, dtype=torch.float64, device=lam.device)
    S = ctypes.c_int64()
    _check(ctx.call(_lib.l1_select, ctx.handle, _ptr(lam), _ptr(sum_lambda), n, int(s_out), seed, cap,
                          _ptr(idx), _ptr(w), ctypes.byref(S)), "l1_select")
    return idx[:S.value], w[:S.value], S.value


def l1_regress_batched(ctx, items, eps=0.05):
    """Solve many instances in one batch (one captured graph).

    items: dicts with A ((d, n) tensor), b, prm (fct_params; s = 0: the
    library's rule) and optionally A_lowp, b_lowp (BF16 copies) and the
    device outputs R_out ((q, q) FP64, column-major), lambda_out ((n,) FP32)
    and idx_out ((cap,) int64).  Returns (results, status):
    results[i] = dict(x, obj, S, s, status)."""
    count = len(items)
    arr = (fct_instance * count)()
    dt = None
    for i, it in enumerate(items):
        n, d, lda = _cm(it["A"])
        lo = it.get("A_lowp")
        ld_lo = _cm(lo)[2] if lo is not None else 0
        io = it.get("idx_out")
        arr[i] = fct_instance(A=_ptr(it["A"]), b=_ptr(it["b"]), A_lowp=_ptr(lo),
                              b_lowp=_ptr(it.get("b_lowp")), n=n, lda=lda, ld_lowp=ld_lo, d=d,
                              pad0=0, prm=it["prm"], R_out=_ptr(it.get("R_out")),
                              lambda_out=_ptr(it.get("lambda_out")), idx_out=_ptr(io),
                              idx_cap=0 if io is None else int(io.numel()))
        t = _dt(it["A"])
        if dt is not None and t != dt:
            raise ValueError("all instances of a batch share one element type")
        dt = t
    total_d = sum(int(it["A"].shape[0]) for it in items)
    x = (ctypes.c_double * total_d)()
    obj = (ctypes.c_double * count)()
    S = (ctypes.c_int64 * count)()
    s_used = (ctypes.c_int32 * count)()
    status = (ctypes.c_int32 * count)()
    st = ctx.call(_lib.l1_regress_batched, ctx.handle, arr, count, dt, eps, x, obj, S, s_used, status)
    if st not in (0, -4, -6, -5) or (st != 0 and all(v == 0 for v in status)):
        _check(st, "l1_regress_batched")
    out, off = [], 0
    for i, it in enumerate(items):
        d = int(it["A"].shape[0])
        out.append(dict(x=list(x[off:off + d]), obj=obj[i], S=S[i], s=s_used[i], status=status[i]))
        off += d
    return out, st


def l1_select_draw(ctx, lam, sum_lambda, s_out, seed, draw, mode, cap):
    """idx, w and S of draw ``draw`` (Bernoulli or with replacement)."""
    n = lam.numel()
    idx = torch.empty(cap, dtype=torch.int64, device=lam.device)
    w = torch.empty(cap, dtype=torch.float64, device=lam.device)
    S = ctypes.c_int64()
    _check(ctx.call(_lib.l1_select_draw, ctx.handle, _ptr(lam), _ptr(sum_lambda), n, int(s_out),
                    seed, int(draw), int(mode), int(cap), _ptr(idx), _ptr(w), ctypes.byref(S)),
           "l1_select_draw")
    return idx, w, S.value


def l1_regress_multi(ctx, A, b, prm, K, mode=FCT_SAMPLE_BERNOULLI, eps=0.05):
    """K draws from one sampling pass and their K solves: (x (K, d) numpy,
    obj, S, status, return status)."""
    import numpy as np
    n, d, lda = _cm(A)
    x = (ctypes.c_double * (K * d))()
    obj = (ctypes.c_double * K)()
    S = (ctypes.c_int64 * K)()
    status = (ctypes.c_int32 * K)()
    st = ctx.call(_lib.l1_regress_multi, ctx.handle, _ptr(A), _ptr(b), n, d, lda, _dt(A), eps,
                  ctypes.byref(prm), int(K), int(mode), x, obj, S, status)
    if st not in (0, -4, -6, -5) or (st != 0 and all(v == 0 for v in status)):
        _check(st, "l1_regress_multi")
    return (np.array(x[:]).reshape(K, d), list(obj), list(S), list(status), st)


def l1_regress_mrhs(ctx, A, B, prm, eps=0.05, R_out=None, lambda_out=None):
    """Multiple l1 regression: A (d, n) and B (k, n) device tensors (column-major
    storage); returns (W (d, k) numpy, obj, S, status, return status).  R_out
    ((q, q) FP64 device, filled column-major) and lambda_out ((n,) FP32) are
    optional."""
    import numpy as np
    n, d, lda = _cm(A)
    nb, k, ldb = _cm(B)
    if nb != n:
        raise ValueError("A and B need the same rows")
    W = (ctypes.c_double * (d * k))()
    obj = (ctypes.c_double * k)()
    S = ctypes.c_int64()
    status = (ctypes.c_int32 * k)()
    st = ctx.call(_lib.l1_regress_mrhs, ctx.handle, _ptr(A), _ptr(B), n, d, k, lda, ldb, _dt(A), eps,
                  ctypes.byref(prm), W, obj, ctypes.byref(S), status, _ptr(R_out), _ptr(lambda_out))
    if st not in (0, -4, -6, -5) or (st != 0 and all(v == 0 for v in status)):
        _check(st, "l1_regress_mrhs")
    return np.array(W[:]).reshape(k, d).T, list(obj), S.value, list(status), st


def l1_subspace(ctx, A, prm, eps=0.05, R_out=None, lambda_out=None):
    """l1 subspace approximation of the rows of A ((d, n) device tensor):
    (W (d, d) numpy with W[j, j] = -1, err (d,), j_star, S, status, return
    status); R_out and lambda_out as for l1_regress_mrhs."""
    import numpy as np
    n, d, lda = _cm(A)
    W = (ctypes.c_double * (d * d))()
    err = (ctypes.c_double * d)()
    js = ctypes.c_int32()
    S = ctypes.c_int64()
    status = (ctypes.c_int32 * d)()
    st = ctx.call(_lib.l1_subspace, ctx.handle, _ptr(A), n, d, lda, _dt(A), eps, ctypes.byref(prm),
                  W, err, ctypes.byref(js), ctypes.byref(S), status, _ptr(R_out), _ptr(lambda_out))
    if st not in (0, -4, -6, -5) or (st != 0 and all(v == 0 for v in status)):
        _check(st, "l1_subspace")
    return np.array(W[:]).reshape(d, d).T, np.array(err[:]), js.value, S.value, list(status), st


def fct_l1_objectives(ctx, A, B, W):
    """sum_i |(A W)_ij - B_ij| for the columns of W ((d, k) numpy); B (k, n) or None."""
    import numpy as np
    n, d, lda = _cm(A)
    W = np.asarray(W, dtype=np.float64)
    k = W.shape[1]
    ldb = _cm(B)[2] if B is not None else n
    Wc = (ctypes.c_double * (d * k))(*W.T.reshape(-1).tolist())
    out = (ctypes.c_double * k)()
    _check(ctx.call(_lib.fct_l1_objectives, ctx.handle, _ptr(A), _ptr(B), n, d, k, lda, ldb, _dt(A),
                    Wc, out), "fct_l1_objectives")
    return np.array(out[:])


def l1_solve(ctx, At, bt, w, iters=0):
    """Weighted l1 solve of a device coreset At (d, S storage)."""
    import numpy as np
    S, d, ldat = _cm(At)
    x = (ctypes.c_double * d)()
    obj = ctypes.c_double()
    _check(ctx.call(_lib.l1_solve, ctx.handle, _ptr(At), _ptr(bt), _ptr(w), S, d, ldat, _dt(At), iters, x,
                         ctypes.byref(obj)), "l1_solve")
    return np.array(x[:], dtype=np.float64), obj.value


def fct_rng_words(ctx, stream, seed, idx0, count, device="cuda"):
    out = torch.empty(4 * count, dtype=torch.int32, device=device)
    _check(ctx.call(_lib.fct_rng_words, ctx.handle, stream, seed, idx0, count, _ptr(out)), "fct_rng_words")
    return out


def fct_pi1_streams(ctx, seed, r1, s, j0, count, device="cuda"):
    bh = torch.empty(count, dtype=torch.int32, device=device)
    ch = torch.empty(count, dtype=torch.float32, device=device)
    bi = torch.empty(count, dtype=torch.int32, device=device)
    ci = torch.empty(count, dtype=torch.float32, device=device)
    sg = torch.empty(count, dtype=torch.int8, device=device)
    _check(ctx.call(_lib.fct_pi1_streams, ctx.handle, seed, r1, s, j0, count, _ptr(bh), _ptr(ch), _ptr(bi),
                                _ptr(ci), _ptr(sg)), "fct_pi1_streams")
    return bh, ch, bi, ci, sg


def fct_fwht(ctx, x, s):
    """In-place normalized FWHT of consecutive s-blocks of a float32 device vector."""
    if x.dtype != torch.float32 or x.numel() % s:
        raise ValueError("float32 tensor with a multiple of s elements expected")
    _check(ctx.call(_lib.fct_fwht, ctx.handle, _ptr(x), x.numel() // s, s), "fct_fwht")
    return x


def fct_to_bf16(ctx, x):
    y = torch.empty(x.shape, dtype=torch.int16, device=x.device)
    _check(ctx.call(_lib.fct_to_bf16, ctx.handle, _ptr(x.contiguous()), x.numel(), _ptr(y)), "fct_to_bf16")
    return y


def fct_lowp_residual(ctx, A, b, R):
    """(r_lowp, R_res): the BF16 residual column b - A x0 (int16 storage) and
    the q x q view of R T for the BF16 sampling pass on [A_lowp, -r0]."""
    n, d, lda = _cm(A)
    q = d + 1
    Rbuf = R.t().contiguous()
    r = torch.empty(n, dtype=torch.int16, device=A.device)
    Rres = torch.empty((q, q), dtype=torch.float64, device=A.device)
    _check(ctx.call(_lib.fct_lowp_residual, ctx.handle, _ptr(A), _ptr(b), n, d, lda, _dt(A),
                    _ptr(Rbuf), _ptr(r), _ptr(Rres)), "fct_lowp_residual")
    return r, Rres.t()


def fct_l1_objective(ctx, A, b, x):
    n, d, lda = _cm(A)
    xs = (ctypes.c_double * d)(*[float(v) for v in x])
    out = ctypes.c_double()
    _check(ctx.call(_lib.fct_l1_objective, ctx.handle, _ptr(A), _ptr(b), n, d, lda, _dt(A), xs,
                                 ctypes.byref(out)), "fct_l1_objective")
    return out.value
