"""Counter-based random streams of the oracle (test infrastructure only).

The paper only asks that the hash columns of B be independent and uniform over
the r1 standard basis vectors, that the diagonal of C hold independent
Cauchy variates (Section "FCT1 Construction"), that Pi2 hold independent
Cauchys (FastCauchyRegression figure, step 3) and that D_ii be an independent
Bernoulli draw (step 7).  It does not name a generator.  This build draws all
of them from Philox4x32-10, the counter-based generator of Salmon, Moraes,
Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11), written
here from that paper's definition:

* state: a 128-bit counter (x0, x1, x2, x3) and a 64-bit key (k0, k1);
* one round: (hi0, lo0) = M0 * x0 and (hi1, lo1) = M1 * x2 as 32x32->64-bit
  products, then (x0, x1, x2, x3) <- (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0);
* the key is bumped by the Weyl constants (W0, W1) between rounds; ten rounds.

Stream layout (a build decision, shared by both sides only through this
written description): key = (seed mod 2^32, seed >> 32); counter =
(idx mod 2^32, idx >> 32, stream, instance).

* stream 0, idx = k >> 1 for stacked position k (the column index of B and C,
  k < 2 n'): words (w0, w1) give the bucket and the Cauchy of the even
  position of the pair, (w2, w3) those of the odd one.  Row j of block
  beta = floor(j / s), t = j mod s, sits at position 2 s beta + t (H-half) and
  2 s beta + s + t (I-half).  Bucket = floor(w * r1 / 2^32).
* stream 1, idx = j >> 7: bit (j & 31) of word (j >> 5) & 3 gives the sign
  D(j) = 1 - 2*bit.
* stream 2, idx = a * r2 + c: word w0 gives the Cauchy Pi2[a, c]; for the
  optimized regression (Gaussian Pi2) words (w0, w1) give the Gaussian
  Pi2[a, c] by the Box-Muller transform.
* stream 3, idx = i >> 2: word (i & 3) is the uniform that decides row i
  (instance k: the k-th of several independent draws from one sampling pass).
* stream 4, idx = j >> 2: word (j & 3) is the uniform of sample j of a draw
  with replacement (instance k: the k-th draw).
* stream 5, idx = g >> 2, g = beta s + k: word (g & 3) picks row
  floor(w t / 2^32) of block beta for sample k of the FCT2 transform's G.
* stream 6, idx = g >> 2, g = i 2^40 + m: word (g & 3) gives the Cauchy
  C[i, m] of FCT2's dense r1 x (n s / t) matrix.  FCT2's signs D are
  stream 1's, like FCT1's.

Pinned by ``tests/test_oracle_rng.py`` against an independent implementation
(rocRAND's Philox4x32-10 engine, compiled on the host) and by distribution
tests.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)

STREAM_PI1 = 0
STREAM_SIGN = 1
STREAM_PI2 = 2
STREAM_SAMPLE = 3
STREAM_REPLACE = 4
STREAM_FCT2_ROWS = 5
STREAM_FCT2_CAUCHY = 6


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Ten Philox4x32 rounds on arrays of 32-bit counter words.

    c0..c3 are broadcastable integer arrays holding values < 2^32; k0, k1 are
    Python ints < 2^32.  Returns four uint32 arrays.
    """
    x0 = np.asarray(c0, dtype=np.uint64) & MASK32
    x1 = np.asarray(c1, dtype=np.uint64) & MASK32
    x2 = np.asarray(c2, dtype=np.uint64) & MASK32
    x3 = np.asarray(c3, dtype=np.uint64) & MASK32
    x0, x1, x2, x3 = np.broadcast_arrays(x0, x1, x2, x3)
    ka, kb = int(k0) & 0xFFFFFFFF, int(k1) & 0xFFFFFFFF
    for _ in range(10):
        p0 = M0 * x0            # exact: both factors < 2^32
        p1 = M1 * x2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        x0, x1, x2, x3 = (hi1 ^ x1 ^ np.uint64(ka), lo1,
                          hi0 ^ x3 ^ np.uint64(kb), lo0)
        ka = (ka + W0) & 0xFFFFFFFF
        kb = (kb + W1) & 0xFFFFFFFF
    return (x0.astype(np.uint32), x1.astype(np.uint32),
            x2.astype(np.uint32), x3.astype(np.uint32))


def stream_words(seed: int, stream: int, idx, instance: int = 0):
    """The four words of call ``idx`` (array) of ``stream`` under ``seed``."""
    idx = np.asarray(idx, dtype=np.uint64)
    seed = int(seed)
    return philox4x32_10(idx & MASK32, idx >> np.uint64(32),
                         np.uint64(stream), np.uint64(instance),
                         seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)


def bucket_from_word(w, r1: int):
    """floor(w * r1 / 2^32): a uniform bucket in [0, r1) (multiply-shift)."""
    return ((np.asarray(w, dtype=np.uint64) * np.uint64(r1)) >> np.uint64(32)).astype(np.int64)


def cauchy_from_word(w):
    """Standard Cauchy variate from a 32-bit word, by inversion, in FP64.

    With u = (w + 1/2) / 2^32 the value is tan(pi (u - 1/2)), the inverse of
    the Cauchy CDF 1/2 + arctan(x)/pi (density 1/(pi (1 + x^2)), Section
    "Preliminaries", sums of Cauchy random variables).  It is evaluated near
    the poles without cancellation: with m = min(w, 2^32 - 1 - w) and
    v = (m + 1/2) / 2^32 in (0, 1/2), the value is -cot(pi v) for w < 2^31 and
    +cot(pi v) otherwise.
    """
    w = np.asarray(w, dtype=np.uint64)
    neg = w < np.uint64(1 << 31)
    m = np.where(neg, w, np.uint64(0xFFFFFFFF) - w).astype(np.float64)
    v = (m + 0.5) / 4294967296.0
    c = 1.0 / np.tan(np.pi * v)
    return np.where(neg, -c, c)


def position_streams(seed: int, k, r1: int, instance: int = 0):
    """(bucket, Cauchy) of stacked positions k (array) of stream 0."""
    k = np.asarray(k, dtype=np.uint64)
    w0, w1, w2, w3 = stream_words(seed, STREAM_PI1, k >> np.uint64(1), instance)
    odd = (k & np.uint64(1)).astype(bool)
    return (bucket_from_word(np.where(odd, w2, w0), r1),
            cauchy_from_word(np.where(odd, w3, w1)))


def row_positions(n_pad: int, s: int, row0: int = 0):
    """Stacked positions of the H-half and I-half copies of padded rows
    j in [row0, row0 + n_pad) (row0 a multiple of s)."""
    j = np.arange(row0, row0 + n_pad, dtype=np.int64)
    kH = 2 * s * (j // s) + j % s
    return kH, kH + s


def pi1_streams(seed: int, n_pad: int, r1: int, s: int, instance: int = 0, row0: int = 0):
    """Per padded row j in [row0, row0 + n_pad): (bucket_H, cauchy_H, bucket_I, cauchy_I)."""
    kH, kI = row_positions(n_pad, s, row0)
    hH, cH = position_streams(seed, kH, r1, instance)
    hI, cI = position_streams(seed, kI, r1, instance)
    return hH, cH, hI, cI


def signs(seed: int, n_pad: int, instance: int = 0, row0: int = 0):
    """D(j) in {+1, -1} for padded rows j in [row0, row0 + n_pad) (stream 1)."""
    c0 = row0 // 128
    ncalls = (row0 + n_pad + 127) // 128 - c0
    words = np.stack(stream_words(seed, STREAM_SIGN, np.arange(c0, c0 + ncalls, dtype=np.uint64),
                                  instance), axis=1)
    j = np.arange(row0, row0 + n_pad, dtype=np.uint64)
    word = words.reshape(-1)[((j >> np.uint64(5)) - np.uint64(4 * c0)).astype(np.int64)].astype(np.uint64)
    bit = (word >> (j & np.uint64(31))) & np.uint64(1)
    return 1.0 - 2.0 * bit.astype(np.float64)


def pi2_matrix(seed: int, q: int, r2: int, instance: int = 0):
    """Pi2 in R^{q x r2}, independent standard Cauchys (stream 2)."""
    idx = np.arange(q * r2, dtype=np.uint64)
    w0 = stream_words(seed, STREAM_PI2, idx, instance)[0]
    return cauchy_from_word(w0).reshape(q, r2)


def gaussian_from_words(w0, w1):
    """Standard Gaussian variate from two 32-bit words, in FP64.

    Box and Muller (1958): for independent uniforms u1, u2 in (0, 1),
    sqrt(-2 ln u1) cos(2 pi u2) is standard normal (the pair (R, Theta) with
    R^2 = -2 ln u1 exponential of mean 2 and Theta uniform is the polar form of
    two independent standard normals).  Here u = (w + 1/2) / 2^32, so u1 is
    never 0 or 1.
    """
    u1 = (np.asarray(w0, dtype=np.float64) + 0.5) / 4294967296.0
    u2 = (np.asarray(w1, dtype=np.float64) + 0.5) / 4294967296.0
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def pi2_gaussian_matrix(seed: int, q: int, r2: int, instance: int = 0):
    """Pi2 in R^{q x r2}, independent standard Gaussians (stream 2, words 0
    and 1): the optimized regression figure's step 4."""
    idx = np.arange(q * r2, dtype=np.uint64)
    w = stream_words(seed, STREAM_PI2, idx, instance)
    return gaussian_from_words(w[0], w[1]).reshape(q, r2)


def sample_words(seed: int, n: int, instance: int = 0, start: int = 0):
    """The uniform 32-bit word deciding each row i in [start, start + n) (stream 3)."""
    i = np.arange(start, start + n, dtype=np.uint64)
    c0 = start >> 2
    ncalls = ((start + n + 3) >> 2) - c0
    words = np.stack(stream_words(seed, STREAM_SAMPLE, np.arange(c0, c0 + ncalls, dtype=np.uint64), instance), axis=1)
    return words.reshape(-1)[(i - np.uint64(4 * c0)).astype(np.int64)]


def replacement_words(seed: int, count: int, instance: int = 0):
    """The uniform 32-bit word of each sample j in [0, count) of a draw with
    replacement (stream 4)."""
    ncalls = (count + 3) >> 2
    words = np.stack(stream_words(seed, STREAM_REPLACE, np.arange(ncalls, dtype=np.uint64), instance), axis=1)
    return words.reshape(-1)[:count]


def fct2_rows(seed: int, nblocks: int, s: int, t: int, instance: int = 0, block0: int = 0):
    """The row of its block (in [0, t)) that FCT2's sample k of block beta
    takes, for blocks [block0, block0 + nblocks): array (nblocks, s)."""
    g = (np.arange(block0, block0 + nblocks, dtype=np.uint64)[:, None] * np.uint64(s)
         + np.arange(s, dtype=np.uint64)[None, :]).reshape(-1)
    words = np.stack(stream_words(seed, STREAM_FCT2_ROWS, g >> np.uint64(2), instance), axis=1)
    w = words[np.arange(g.size), (g & np.uint64(3)).astype(np.int64)].astype(np.uint64)
    return ((w * np.uint64(t)) >> np.uint64(32)).astype(np.int64).reshape(nblocks, s)


def fct2_cauchy(seed: int, r1: int, m0: int, count: int, instance: int = 0):
    """FCT2's C[i, m] for i < r1 and m in [m0, m0 + count): array (r1, count)."""
    i = np.arange(r1, dtype=np.uint64)[:, None]
    m = np.arange(m0, m0 + count, dtype=np.uint64)[None, :]
    g = ((i << np.uint64(40)) | m).reshape(-1)
    words = np.stack(stream_words(seed, STREAM_FCT2_CAUCHY, g >> np.uint64(2), instance), axis=1)
    w = words[np.arange(g.size), (g & np.uint64(3)).astype(np.int64)]
    return cauchy_from_word(w).reshape(r1, count)
