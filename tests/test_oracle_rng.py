"""Pins of the oracle's random streams (CPU only).

* Philox4x32-10 against rocRAND's engine compiled for the host (an
  independent implementation of the same published generator);
* bucket uniformity (chi-square), Cauchy law (Kolmogorov-Smirnov against the
  CDF 1/2 + arctan(x)/pi, the density of the preliminaries section), the
  median of |Cauchy| equal to tan(pi/4) = 1, and closed forms at edge words;
* sign and sampling words balanced.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.stats

from oracle import philox

HERE = os.path.dirname(os.path.abspath(__file__))


def _ref_binary(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available for the rocRAND host reference")
    out = tmp_path_factory.mktemp("rng") / "philox_ref"
    src = os.path.join(HERE, "rng_ref", "philox_ref.cpp")
    r = subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", "-I/opt/rocm/include",
                        src, "-o", str(out)], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("could not build rocRAND host reference: " + r.stderr[-400:])
    return str(out)


def test_philox_matches_rocrand_host_engine(tmp_path_factory):
    exe = _ref_binary(tmp_path_factory)
    g = np.random.default_rng(5)
    cases = [(0, 0, 0, 0, 0), (2**64 - 1, 2**32 - 1, 2**30 - 1, 2**32 - 1, 2**32 - 1),
             (0, 1, 0, 0, 0), (1, 0, 0, 3, 7)]
    for _ in range(200):
        cases.append((int(g.integers(0, 2**63)), int(g.integers(0, 2**32)), int(g.integers(0, 2**30)),
                      int(g.integers(0, 4)), int(g.integers(0, 300))))
    inp = "\n".join(" ".join(str(v) for v in c) for c in cases) + "\n"
    r = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True)
    ref = np.array([[int(t) for t in line.split()] for line in r.stdout.strip().splitlines()], dtype=np.uint64)
    seeds = np.array([c[0] for c in cases], dtype=np.uint64)
    c = np.array([c[1:] for c in cases], dtype=np.uint64)
    got = np.empty_like(ref)
    for i, s in enumerate(seeds):
        s = int(s)
        w = philox.philox4x32_10(c[i, 0], c[i, 1], c[i, 2], c[i, 3], s & 0xFFFFFFFF, s >> 32)
        got[i] = [int(x) for x in w]
    assert np.array_equal(got, ref)


def test_buckets_uniform_chi2():
    r1 = 97
    h = philox.pi1_streams(11, 1 << 16, r1, 256)[0]
    assert h.min() >= 0 and h.max() < r1
    counts = np.bincount(h, minlength=r1)
    chi2, pval = scipy.stats.chisquare(counts)
    assert pval > 1e-4


def test_bucket_multiply_shift_edges():
    w = np.array([0, 1, 2**31, 2**32 - 1], dtype=np.uint64)
    assert list(philox.bucket_from_word(w, 2048)) == [0, 0, 1024, 2047]
    assert list(philox.bucket_from_word(w, 1)) == [0, 0, 0, 0]


def test_cauchy_law_ks_and_median():
    words = np.concatenate(philox.stream_words(3, philox.STREAM_PI1, np.arange(50000)))
    c = philox.cauchy_from_word(words)
    ks = scipy.stats.kstest(c, lambda x: 0.5 + np.arctan(x) / np.pi)
    assert ks.pvalue > 1e-4
    assert abs(np.median(np.abs(c)) - 1.0) < 0.02          # tan(pi/4)
    assert abs(np.mean(c > 0) - 0.5) < 0.01


def test_cauchy_edge_words_closed_form():
    w = np.array([0, 2**31 - 1, 2**31, 2**32 - 1, 2**30], dtype=np.uint64)
    c = philox.cauchy_from_word(w)
    eps = np.pi * 2.0**-33
    # w = 0: u = 2^-33, tan(pi(u - 1/2)) = -cot(pi 2^-33) ~ -1/eps
    assert np.isclose(c[0], -1.0 / np.tan(eps), rtol=1e-12)
    assert np.isclose(c[1], -np.tan(eps), rtol=1e-9)          # just below the centre
    assert np.isclose(c[2], np.tan(eps), rtol=1e-9)           # just above the centre
    assert np.isclose(c[3], 1.0 / np.tan(eps), rtol=1e-12)
    # w = 2^30: u = (2^30 + 1/2)/2^32 ~ 1/4, tan(-pi/4 + tiny) ~ -1
    assert np.isclose(c[4], np.tan(np.pi * ((2**30 + 0.5) / 2**32 - 0.5)), rtol=1e-12)
    # matches scipy's quantile function away from the poles
    g = np.random.default_rng(0).integers(2**20, 2**32 - 2**20, size=1000, dtype=np.uint64)
    u = (g.astype(np.float64) + 0.5) / 2.0**32
    assert np.allclose(philox.cauchy_from_word(g), scipy.stats.cauchy.ppf(u), rtol=1e-9, atol=1e-12)


def test_signs_and_sampling_words_balanced():
    d = philox.signs(9, 1 << 16)
    assert set(np.unique(d)) == {-1.0, 1.0}
    assert abs(d.mean()) < 0.02
    # signs of consecutive rows come from distinct bits (no block repetition)
    assert not np.array_equal(d[:128], d[128:256])
    u = philox.sample_words(9, 1 << 16).astype(np.float64) / 2.0**32
    assert scipy.stats.kstest(u, "uniform").pvalue > 1e-4
    # an offset window agrees with the full stream
    assert np.array_equal(philox.sample_words(9, 37, start=101), philox.sample_words(9, 200)[101:138])


def test_position_pairs_share_a_call():
    # positions 2c and 2c+1 use words (w0, w1) and (w2, w3) of call c
    w = philox.stream_words(4, 0, np.arange(10))
    h, c = philox.position_streams(4, np.arange(20), 64)
    assert np.array_equal(h[0::2], philox.bucket_from_word(w[0], 64))
    assert np.array_equal(h[1::2], philox.bucket_from_word(w[2], 64))
    assert np.array_equal(c[1::2], philox.cauchy_from_word(w[3]))
    kH, kI = philox.row_positions(12, 4)
    assert list(kH) == [0, 1, 2, 3, 8, 9, 10, 11, 16, 17, 18, 19]
    assert list(kI) == [4, 5, 6, 7, 12, 13, 14, 15, 20, 21, 22, 23]


def test_streams_and_instances_independent():
    a = philox.stream_words(1, 0, np.arange(64))[0]
    b = philox.stream_words(1, 1, np.arange(64))[0]
    c = philox.stream_words(1, 0, np.arange(64), instance=1)[0]
    assert not np.array_equal(a, b) and not np.array_equal(a, c)


def test_windowed_streams_are_slices_of_the_whole():
    full = philox.pi1_streams(6, 4096, 50, 64)
    win = philox.pi1_streams(6, 1024, 50, 64, row0=2048)
    for a, b in zip(full, win):
        assert np.array_equal(a[2048:3072], b)
    assert np.array_equal(philox.signs(6, 4096)[1280:1280 + 700], philox.signs(6, 700, row0=1280))
