"""Pins of the oracle's FCT1 (CPU only).

* H_s from the Sylvester recursion equals scipy's Hadamard construction and
  the printed H_2; H_s H_s = I; the butterfly FWHT equals the dense matrix;
* Pi1 X computed fast equals Pi1 built as the explicit product 4 B C H~ D
  (both sign modes, n not a multiple of s);
* exact invariants from the FCT1 proof: ||G_s z||_2^2 = 2 ||z||_2^2, the
  uncertainty bound ||G_s z||_1 >= s^(1/4) ||z||_2 / 2, and conservation of
  the column sums when every Cauchy is 1 (B has one 1 per column and
  1^T H_s = sqrt(s) e_0^T);
* linearity and zero padding;
* 1-stability: a column sum of Pi1 x is Cauchy with scale 4 ||H~ x||_1.
"""
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.stats

from oracle import fct, philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_hadamard_matches_printed_h2_and_scipy():
    h2 = np.loadtxt(os.path.join(GOLDEN, "hadamard_h2.txt"))
    assert np.array_equal(fct.hadamard_sylvester(2) * np.sqrt(2), h2)
    for s in (1, 2, 4, 8, 16, 32, 64, 256):
        H = fct.hadamard_sylvester(s)
        assert np.allclose(H, scipy.linalg.hadamard(s) / np.sqrt(s), atol=0)
        assert np.allclose(H @ H, np.eye(s), atol=1e-13)


@pytest.mark.parametrize("s", [2, 4, 8, 16, 32, 64])
def test_fwht_equals_dense(s):
    z = np.random.default_rng(s).standard_normal((5, s, 3))
    got = fct.fwht_blocks(z)
    H = scipy.linalg.hadamard(s) / np.sqrt(s)
    ref = np.einsum("ij,bjq->biq", H, z)
    assert np.max(np.abs(got - ref)) <= 1e-14 * max(1.0, np.abs(z).sum())


@pytest.mark.parametrize("sign_flip", [False, True])
@pytest.mark.parametrize("s,n,r1", [(2, 9, 3), (4, 16, 5), (8, 37, 16), (16, 70, 7), (16, 256, 16)])
def test_pi1_fast_equals_dense(s, n, r1, sign_flip):
    X = np.random.default_rng(n).standard_normal((n, 3))
    P = fct.pi1_dense(n, s, r1, seed=42, sign_flip=sign_flip)
    assert P.shape == (r1, n)
    fast = fct.pi1_apply(X, s, r1, seed=42, sign_flip=sign_flip)
    assert np.max(np.abs(fast - P @ X)) <= 1e-12 * np.abs(P).sum(axis=1).max() * np.abs(X).max()


def test_dense_pi1_has_paper_structure():
    # without signs, every column of 4^-1 Pi1 restricted to one block is a
    # sum of Cauchy-weighted basis vectors: B has exactly one 1 per column.
    n, s, r1 = 8, 4, 5
    P = fct.pi1_dense(n, s, r1, seed=1, sign_flip=False)
    hH, cH, hI, cI = philox.pi1_streams(1, n, r1, s)
    # column 0 of block 0: H-half rows contribute cH[t] * H[t, 0] = cH[t]/sqrt(s) into hH[t],
    # and the I-half contributes cI[0] into hI[0].
    col = np.zeros(r1)
    for t in range(s):
        col[hH[t]] += 4 * cH[t] / np.sqrt(s)
    col[hI[0]] += 4 * cI[0]
    assert np.allclose(P[:, 0], col, rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("s", [4, 16, 64, 256])
def test_stacked_block_norm_and_uncertainty(s):
    G = np.vstack([fct.hadamard_sylvester(s), np.eye(s)])
    H = scipy.linalg.hadamard(s) / np.sqrt(s)
    zs = [np.eye(s)[0], H[:, 3], H[:, s - 1] + np.eye(s)[1],
          np.random.default_rng(s).standard_normal(s)]
    for z in zs:
        gz = G @ z
        assert np.isclose(gz @ gz, 2 * (z @ z), rtol=1e-12)
        assert np.abs(gz).sum() >= 0.5 * s**0.25 * np.linalg.norm(z) - 1e-12
        assert np.abs(gz).sum() <= np.sqrt(4 * s) * np.abs(z).sum() + 1e-12


def test_conservation_with_unit_cauchys():
    n, s, r1 = 1000, 16, 32
    X = np.random.default_rng(2).standard_normal((n, 2))
    Y = fct.pi1_apply(X, s, r1, seed=3, sign_flip=False, cauchy_one=True)
    n_pad = fct.padded_rows(n, s)
    Z = np.zeros((n_pad, 2))
    Z[:n] = X
    blocks = Z.reshape(-1, s, 2)
    expect = 4 * (np.sqrt(s) * blocks[:, 0, :] + blocks.sum(axis=1)).sum(axis=0)
    assert np.allclose(Y.sum(axis=0), expect, rtol=1e-12)


def test_linearity_and_zero_padding():
    g = np.random.default_rng(4)
    X1, X2 = g.standard_normal((300, 3)), g.standard_normal((300, 3))
    a, b = 2.5, -0.75
    Y = lambda X: fct.pi1_apply(X, 32, 24, seed=9)
    assert np.allclose(Y(a * X1 + b * X2), a * Y(X1) + b * Y(X2), rtol=1e-11, atol=1e-9)
    # appending zero rows inside the padding changes nothing
    Xz = np.vstack([X1, np.zeros((20, 3))])
    assert np.allclose(Y(Xz), Y(X1), rtol=0, atol=0)
    # duplicate columns give duplicate outputs
    Yd = Y(np.hstack([X1[:, :1], X1[:, :1]]))
    assert np.array_equal(Yd[:, 0], Yd[:, 1])


def test_column_sum_is_cauchy_with_l1_scale():
    # sum_i (Pi1 x)_i = 4 sum_k C(k) g_k, a Cauchy scaled by 4 ||g||_1 (1-stability)
    n, s, r1 = 64, 16, 8
    x = np.random.default_rng(7).standard_normal((n, 1))
    g = np.vstack([fct.hadamard_sylvester(s), np.eye(s)])
    gl1 = sum(np.abs(g @ x[s * i: s * (i + 1), 0]).sum() for i in range(n // s))
    vals = np.array([fct.pi1_apply(x, s, r1, seed=sd, sign_flip=False).sum() for sd in range(600)])
    z = vals / (4 * gl1)
    assert scipy.stats.kstest(z, lambda t: 0.5 + np.arctan(t) / np.pi).pvalue > 1e-3


def test_row_scale_bounds_result():
    X = np.random.default_rng(5).standard_normal((500, 4))
    Y, S = fct.pi1_apply(X, 16, 20, seed=1, return_scale=True)
    assert np.all(np.abs(Y).max(axis=1) <= S * (1 + 1e-12))


def test_row_windows_add_up_to_the_whole():
    # Pi1 acts block by block and the streams are indexed by the global row, so
    # the sketches of consecutive windows (global offsets) sum to the sketch of
    # the whole design; each window equals the columns of dense Pi1 it touches.
    n, s, r1 = 1000, 16, 24
    X = np.random.default_rng(8).standard_normal((n, 3))
    whole = fct.pi1_apply(X, s, r1, seed=5)
    cuts = [0, 256, 512, 768, n]
    parts = sum(fct.pi1_apply(X[a:b], s, r1, seed=5, row0=a) for a, b in zip(cuts[:-1], cuts[1:]))
    assert np.allclose(parts, whole, rtol=1e-12, atol=1e-12 * np.abs(whole).max())
    P = fct.pi1_dense(n, s, r1, seed=5)
    assert np.allclose(fct.pi1_apply(X[256:512], s, r1, seed=5, row0=256), P[:, 256:512] @ X[256:512],
                       rtol=1e-12, atol=1e-10)
    with pytest.raises(ValueError):
        fct.pi1_apply(X[:40], s, r1, seed=5, row0=8)
