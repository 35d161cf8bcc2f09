"""FCT1, the Fast Cauchy Transform Pi1 = 4 B C H~ (test infrastructure only).

Section "FCT1 Construction: via a Low-coherence Matrix" defines

* H~ in R^{2n x n}: block diagonal with n/s blocks G_s = [H_s ; I_s], H_s the
  normalized s x s Hadamard matrix (Sylvester recursion
  H_n = [[H_{n/2}, H_{n/2}], [H_{n/2}, -H_{n/2}]], H_2 = [[1, 1], [1, -1]],
  normalized by 1/sqrt(n));
* C in R^{2n x 2n}: diagonal, independent standard Cauchys;
* B in R^{r1 x 2n}: each column an independent uniform standard basis vector;
* the factor 4.

Readings taken here (each is listed with its reason in the design notes):

* n need not be a multiple of s: X is padded with zero rows to
  n' = s * ceil(n / s);
* inside block beta the H-half rows come first: stacked position
  2 s beta + t holds (H_s z_beta)_t and 2 s beta + s + t holds (z_beta)_t;
* an optional random sign diagonal D (row j multiplied by D(j)) is applied
  before H~; with ``sign_flip=False`` Pi1 is exactly the paper's.

``pi1_apply`` computes Pi1 X with a butterfly Walsh-Hadamard transform and
per-column bucket sums; ``pi1_dense`` builds Pi1 as an explicit matrix for
tiny n from the Kronecker recursion.  They share only the random streams.
"""
from __future__ import annotations

import numpy as np

from . import philox


def hadamard_sylvester(s: int) -> np.ndarray:
    """Normalized s x s Hadamard matrix from the Sylvester recursion (FCT1 section)."""
    if s < 1 or s & (s - 1):
        raise ValueError("s must be a power of two")
    h = np.array([[1.0]])
    h2 = np.array([[1.0, 1.0], [1.0, -1.0]])
    while h.shape[0] < s:
        h = np.kron(h2, h)          # [[H, H], [H, -H]]
    return h / np.sqrt(s)


def fwht_blocks(z: np.ndarray) -> np.ndarray:
    """Normalized Walsh-Hadamard transform along axis 1 of z (nb, s, q).

    Radix-2 butterflies in Sylvester (natural) order: at span h, entries i and
    i + h of every 2h-group become (a + b, a - b).  Divided by sqrt(s) once.
    """
    z = np.array(z, dtype=np.float64, copy=True)
    nb, s, q = z.shape
    h = 1
    while h < s:
        v = z.reshape(nb, s // (2 * h), 2, h, q)
        a = v[:, :, 0].copy()
        b = v[:, :, 1]
        v[:, :, 0] = a + b
        v[:, :, 1] = a - b
        h *= 2
    return z / np.sqrt(s)


def padded_rows(n: int, s: int) -> int:
    return s * ((n + s - 1) // s)


def pi1_apply(X, s: int, r1: int, seed: int, sign_flip: bool = True,
              instance: int = 0, cauchy_one: bool = False, return_scale: bool = False,
              row0: int = 0, scale_per_column: bool = False):
    """Y = Pi1 X in FP64 for X of shape (n, q).

    ``cauchy_one`` replaces every Cauchy by 1 (used by conservation pins).
    ``return_scale`` also returns, per output row i, the l1 mass of the fully
    expanded sum that forms it: S_i = max_j sum_{k: h(k)=i} 4 |C(k)| (|G_s| |z|)_kj,
    where |G_s| |z| is sum_v |z_v| / sqrt(s) on the H-half and |z_t| on the
    I-half.  Rounding errors of any evaluation order are bounded relative to
    this scale (a reading of "relative to each output row's scale": |Y_ij|
    itself can cancel, and so can a single (H_s z)_t).
    ``row0`` (a multiple of s) places X as rows [row0, row0 + n) of a larger
    design: every random stream is indexed by the global row, so the results
    of consecutive windows add up to Pi1 of their union.  With
    ``scale_per_column`` the scale comes back before the max over j, as the
    (r1, q) array of masses, which also adds up over windows.
    """
    if row0 % s:
        raise ValueError("row0 must be a multiple of s")
    X = np.asarray(X, dtype=np.float64)
    n, q = X.shape
    n_pad = padded_rows(n, s)
    nb = n_pad // s
    z = np.zeros((n_pad, q))
    z[:n] = X
    if sign_flip:
        z *= philox.signs(seed, n_pad, instance, row0)[:, None]
    hz = fwht_blocks(z.reshape(nb, s, q)).reshape(n_pad, q)
    hH, cH, hI, cI = philox.pi1_streams(seed, n_pad, r1, s, instance, row0)
    if cauchy_one:
        cH = np.ones_like(cH)
        cI = np.ones_like(cI)
    Y = np.zeros((r1, q))
    S = np.zeros((r1, q))
    if return_scale:
        absmass = np.repeat(np.abs(z).reshape(nb, s, q).sum(axis=1), s, axis=0) / np.sqrt(s)
    for col in range(q):
        gH = 4.0 * cH * hz[:, col]
        gI = 4.0 * cI * z[:, col]
        Y[:, col] = (np.bincount(hH, weights=gH, minlength=r1)
                     + np.bincount(hI, weights=gI, minlength=r1))
        if return_scale:
            S[:, col] = (np.bincount(hH, weights=4.0 * np.abs(cH) * absmass[:, col], minlength=r1)
                         + np.bincount(hI, weights=np.abs(gI), minlength=r1))
    if return_scale:
        return Y, (S if scale_per_column else S.max(axis=1))
    return Y


def pi1_dense(n: int, s: int, r1: int, seed: int, sign_flip: bool = True,
              instance: int = 0) -> np.ndarray:
    """Pi1 = 4 B C H~ D as an explicit r1 x n matrix (tiny n only)."""
    n_pad = padded_rows(n, s)
    nb = n_pad // s
    Hs = hadamard_sylvester(s)
    G = np.vstack([Hs, np.eye(s)])                      # G_s = [H_s; I_s]
    Ht = np.zeros((2 * n_pad, n_pad))
    for beta in range(nb):
        Ht[2 * s * beta: 2 * s * (beta + 1), s * beta: s * (beta + 1)] = G
    hH, cH, hI, cI = philox.pi1_streams(seed, n_pad, r1, s, instance)
    bucket = np.empty(2 * n_pad, dtype=np.int64)
    cauchy = np.empty(2 * n_pad)
    for beta in range(nb):
        rows = np.arange(s * beta, s * (beta + 1))
        bucket[2 * s * beta + np.arange(s)] = hH[rows]
        cauchy[2 * s * beta + np.arange(s)] = cH[rows]
        bucket[2 * s * beta + s + np.arange(s)] = hI[rows]
        cauchy[2 * s * beta + s + np.arange(s)] = cI[rows]
    B = np.zeros((r1, 2 * n_pad))
    B[bucket, np.arange(2 * n_pad)] = 1.0
    C = np.diag(cauchy)
    D = np.diag(philox.signs(seed, n_pad, instance) if sign_flip else np.ones(n_pad))
    P = 4.0 * B @ C @ Ht @ D
    return P[:, :n]


def fct2_scale(r1: int, s: int, t: int) -> float:
    """The constant of FCT2 (section "FCT2 Construction"): 8/r1 sqrt(pi t / (2 s))."""
    return 8.0 / r1 * np.sqrt(np.pi * t / (2.0 * s))


def fct2_apply(X, t: int, s: int, r1: int, seed: int, instance: int = 0,
               return_scale: bool = False, row0: int = 0, scale_per_column: bool = False):
    """Y = Pi1 X for FCT2 (section "FCT2 Construction"), FP64:
    Pi1 = 8/r1 sqrt(pi t/(2 s)) C Hbar, Hbar block-diagonal with n'/t blocks
    G = sqrt(t/s) P H_t D (H_t the normalized Sylvester Hadamard of size t, D
    random signs, P keeping s rows drawn uniformly, with replacement, from t;
    the paper only asks G to be a fast Johnson-Lindenstrauss matrix, this is
    the choice), C an r1 x (n' s / t) matrix of independent standard Cauchys.
    Rows are zero-padded to n' = t ceil(n / t).  ``return_scale`` also
    returns S_i = max_j 8/r1 sqrt(pi t/(2 s)) sum_m |C_im| sum_v |x_vj| /
    sqrt(s) (v over the block of m), the magnitude the rounding of any
    evaluation order is bounded by (``scale_per_column``: the (r1, q) masses
    before the max, which add up over row windows).  ``row0`` (a multiple of
    t) places X at global row row0: the streams are indexed by global block
    and row."""
    if row0 % t:
        raise ValueError("row0 must be a multiple of t")
    X = np.asarray(X, dtype=np.float64)
    n, q = X.shape
    n_pad = padded_rows(n, t)
    nb = n_pad // t
    z = np.zeros((n_pad, q))
    z[:n] = X
    z *= philox.signs(seed, n_pad, instance, row0)[:, None]
    hz = fwht_blocks(z.reshape(nb, t, q))                 # (nb, t, q), H_t z
    rows = philox.fct2_rows(seed, nb, s, t, instance, row0 // t)
    Z = np.sqrt(t / s) * hz[np.arange(nb)[:, None], rows]  # (nb, s, q)
    Z = Z.reshape(nb * s, q)
    C = philox.fct2_cauchy(seed, r1, (row0 // t) * s, nb * s, instance)
    c = fct2_scale(r1, s, t)
    Y = c * (C @ Z)
    if not return_scale:
        return Y
    absblk = np.abs(z).reshape(nb, t, q).sum(axis=1) / np.sqrt(s)     # (nb, q)
    zeta = np.repeat(absblk, s, axis=0)                                 # (nb s, q)
    S = c * (np.abs(C) @ zeta)
    return Y, (S if scale_per_column else S.max(axis=1))


def fct2_dense(n: int, t: int, s: int, r1: int, seed: int, instance: int = 0) -> np.ndarray:
    """Pi1 of FCT2 built entry by entry from its definition (small n)."""
    n_pad = padded_rows(n, t)
    nb = n_pad // t
    D = philox.signs(seed, n_pad, instance)
    H = hadamard_sylvester(t)  # normalized
    rows = philox.fct2_rows(seed, nb, s, t, instance)
    Hbar = np.zeros((nb * s, n_pad))
    for beta in range(nb):
        G = np.sqrt(t / s) * H[rows[beta]] * D[beta * t:(beta + 1) * t][None, :]
        Hbar[beta * s:(beta + 1) * s, beta * t:(beta + 1) * t] = G
    C = philox.fct2_cauchy(seed, r1, 0, nb * s, instance)
    return (fct2_scale(r1, s, t) * C @ Hbar)[:, :n]
