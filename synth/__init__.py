"""Seeded synthetic workloads for the l1-regression hot path.

This module only draws inputs; it holds none of the method's arithmetic.  Both
the HIP path (through its tests and the benchmark) and the CPU oracle read the
same bytes it produces.

Every workload follows the structure of the paper's synthetic tests: a dense
design with columns of very different scales and a few high-leverage rows, a
planted x*, Laplace or Gaussian noise, and a fraction of responses replaced by
heavy-tailed (Cauchy) outliers (Section "Empirical Evaluation": the small- and
medium-scale regression test with corrupted responses, and the large-scale
test with imbalanced rows and 0.1% corrupted measurements).  The paper's real
datasets are not used.

Generation is chunked: rows [c 2^20, (c+1) 2^20) are drawn from
``numpy.random.default_rng(SeedSequence([seed, tag, c]))``, so the bytes do not
depend on how many workers generate them.  Values are drawn in FP64 and cast
to the workload dtype; b is formed from the cast A in FP64 and then cast.
Arrays are column-major: ``A`` has shape (d, n) and row ``A[j]`` is column j
of the n x d design.
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

CHUNK = 1 << 20


@dataclass
class Workload:
    name: str
    n: int
    d: int
    dtype: str               # "f32" or "f64"
    s: int                   # FWHT block size
    r1: int                  # sketch rows
    r2: int                  # columns of Pi2
    s_out: int               # expected coreset size
    eps: float               # stated acceptance target
    seed: int = 0
    col_scale_log10: float = 3.0     # columns scaled by 10^U(-a, a); 0 = unscaled
    leverage_frac: float = 0.0       # fraction of rows multiplied by leverage_mult
    leverage_mult: float = 1.0
    noise: str = "laplace"           # "laplace" or "normal"
    noise_scale: float = 0.1
    outlier_frac: float = 0.02
    outlier_scale: float = 1e3
    extra: dict = field(default_factory=dict)

    @property
    def np_dtype(self):
        return np.float64 if self.dtype == "f64" else np.float32


def _rng(seed: int, tag: int, chunk: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([seed, tag, chunk]))


def _chunks(n: int):
    return [(c, c * CHUNK, min(n, (c + 1) * CHUNK)) for c in range((n + CHUNK - 1) // CHUNK)]


def _pick(n: int, count: int, seed: int, tag: int) -> np.ndarray:
    """Exactly ``count`` distinct rows, chosen by a seeded permutation."""
    if count <= 0:
        return np.zeros(0, dtype=np.int64)
    g = np.random.default_rng(np.random.SeedSequence([seed, tag]))
    if n <= (1 << 24):
        return np.sort(g.permutation(n)[:count])
    # large n: rejection-free sample of distinct indices
    got = np.unique(g.integers(0, n, size=int(count * 1.1) + 16))
    while got.size < count:
        got = np.unique(np.concatenate([got, g.integers(0, n, size=count)]))
    return np.sort(g.permutation(got)[:count])


def chunk_context(w: Workload):
    """What every chunk of workload w shares: x*, the column scales, and the
    (sorted) high-leverage and outlier rows of the whole design."""
    g0 = np.random.default_rng(np.random.SeedSequence([w.seed, 0]))
    x_star = g0.standard_normal(w.d)
    if w.col_scale_log10 > 0:
        scale = 10.0 ** g0.uniform(-w.col_scale_log10, w.col_scale_log10, size=w.d)
    else:
        scale = np.ones(w.d)
    lev = _pick(w.n, int(round(w.leverage_frac * w.n)), w.seed, 11)
    out = _pick(w.n, int(round(w.outlier_frac * w.n)), w.seed, 12)
    return x_star, scale, lev, out


def generate_chunk(w: Workload, c: int, ctx=None):
    """Rows [c 2^20, (c+1) 2^20) of workload w: (A (d, rows), b (rows,)),
    the same bytes generate() puts there."""
    x_star, scale, lev, out = ctx if ctx is not None else chunk_context(w)
    lo, hi = c * CHUNK, min(w.n, (c + 1) * CHUNK)
    dt = w.np_dtype
    g = _rng(w.seed, 1, c)
    blk = g.standard_normal((hi - lo, w.d)) * scale
    sel = lev[(lev >= lo) & (lev < hi)] - lo
    blk[sel] *= w.leverage_mult
    Ac = blk.astype(dt)
    if w.noise == "normal":
        eps = g.normal(0.0, w.noise_scale, size=hi - lo)
    else:
        eps = g.laplace(0.0, w.noise_scale, size=hi - lo)
    bc = Ac.astype(np.float64) @ x_star + eps
    sel = out[(out >= lo) & (out < hi)] - lo
    go = _rng(w.seed, 2, c)
    bc[sel] = w.outlier_scale * go.standard_cauchy(sel.size)
    return np.ascontiguousarray(Ac.T), bc.astype(dt)


def generate(w: Workload, threads: int = 8):
    """Return (A (d, n) column-major, b (n,), x_star (d,)) for workload ``w``."""
    ctx = chunk_context(w)
    A = np.empty((w.d, w.n), dtype=w.np_dtype)
    b = np.empty(w.n, dtype=w.np_dtype)

    def work(chunk):
        c, lo, hi = chunk
        A[:, lo:hi], b[lo:hi] = generate_chunk(w, c, ctx)

    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        list(ex.map(work, _chunks(w.n)))
    return A, b, ctx[0]


def separable(n: int, d: int, seed: int = 0, outlier_frac: float = 0.001, dtype=np.float32):
    """Canonical-row design of the paper's large-scale test.

    Row i of A is the canonical vector e_c(i); coordinate c receives about
    twice as many rows as coordinate c + 1; b_i = x*_c(i) + Laplace noise,
    and a fraction of rows is replaced by 1000 times its noise.  Returns
    (A (d, n) column-major, b, coord, x_star).
    """
    g = np.random.default_rng(np.random.SeedSequence([seed, 7]))
    x_star = g.standard_normal(d)
    wts = 2.0 ** -np.arange(d)
    coord = np.sort(g.choice(d, size=n, p=wts / wts.sum()))
    coord = g.permutation(coord)
    eps = g.laplace(0.0, 1.0, size=n)
    bad = g.random(n) < outlier_frac
    b = np.where(bad, 1000.0 * eps, x_star[coord] + eps)
    A = np.zeros((d, n), dtype=dtype)
    A[coord, np.arange(n)] = 1.0
    return A, b.astype(dtype), coord, x_star


# The five workloads of the benchmark configuration list (readings of the
# unstated parameters are documented in the design notes).
SMALL = Workload("small-65536x16-f64", n=65536, d=16, dtype="f64", s=64, r1=512, r2=8,
                 s_out=2000, eps=0.05, col_scale_log10=0.0, noise="normal",
                 noise_scale=0.01, outlier_frac=0.01, outlier_scale=100.0)
TALL = Workload("tall-4194304x32-f32", n=4194304, d=32, dtype="f32", s=256, r1=2048, r2=16,
                s_out=8000, eps=0.05, leverage_frac=0.001, leverage_mult=1e4,
                outlier_frac=0.02, outlier_scale=1e3)
PRECISION = Workload("precision-33554432x64-f32-bf16", n=33554432, d=64, dtype="f32", s=512,
                     r1=4096, r2=24, s_out=20000, eps=0.05, leverage_frac=0.001,
                     leverage_mult=1e4, outlier_frac=0.02, outlier_scale=1e3)
LARGE = Workload("large-268435456x16-f32", n=268435456, d=16, dtype="f32", s=1024, r1=1024,
                 r2=16, s_out=10000, eps=0.01, leverage_frac=0.0001, leverage_mult=1e5,
                 outlier_frac=0.05, outlier_scale=1e4)


def batch_instances(count: int = 256, base_seed: int = 0):
    """The batching workload: per instance n ~ U_int[2^14, 2^20], d in {8,16,32,64}."""
    out = []
    for i in range(count):
        g = np.random.default_rng(np.random.SeedSequence([base_seed + i, 99]))
        n = int(g.integers(1 << 14, (1 << 20) + 1))
        d = int(g.choice([8, 16, 32, 64]))
        r1 = 8 * d * int(np.ceil(np.log2(d)))
        q = d + 1
        out.append(Workload(f"batch-{i}", n=n, d=d, dtype="f32", s=256, r1=r1, r2=16,
                            s_out=250 * q, eps=0.05, seed=base_seed + i, leverage_frac=0.001,
                            leverage_mult=1e4, outlier_frac=0.02, outlier_scale=1e3))
    return out


def scaled(w: Workload, n: int, **kw) -> Workload:
    """Same generator and parameters at another row count (for tests)."""
    from dataclasses import replace
    return replace(w, n=n, name=f"{w.name}@{n}", **kw)
