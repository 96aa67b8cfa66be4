"""Pins for the oracle's random streams (CPU only)."""
import os

import numpy as np
import pytest
from scipy import stats

from oracle import streams


def _rows(path):
    with open(path) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def test_philox_known_answers(golden_dir):
    for row in _rows(os.path.join(golden_dir, "philox4x32_10_kat.txt")):
        v = [int(x, 16) for x in row]
        out = streams.philox4x32_10(*v[:6])
        assert [int(o) for o in out] == v[6:10]


def test_splitmix64_known_answers(golden_dir):
    want = [int(r[0], 16) for r in _rows(os.path.join(golden_dir,
                                                     "splitmix64_kat.txt"))]
    assert streams.splitmix64_sequence(0, len(want)) == want


def test_poly_hash_matches_direct_powers():
    # Horner evaluation vs the polynomial written with explicit powers
    co = streams.hash_coeffs(12345, streams.STREAM_BUCKET)
    assert all(0 <= a < streams.P61 for a in co)
    idx = [0, 1, 2, 3, 1000, 2**31 - 1, 2**40 + 7, 2**60]
    got = streams.poly_hash(co, idx)
    for i, g in zip(idx, got):
        direct = (co[3] * i**3 + co[2] * i**2 + co[1] * i + co[0]) % (2**61 - 1)
        assert int(g) == direct


def test_streams_differ_and_seed_matters():
    a = streams.hash_coeffs(1, streams.STREAM_BUCKET)
    b = streams.hash_coeffs(1, streams.STREAM_SIGN)
    c = streams.hash_coeffs(2, streams.STREAM_BUCKET)
    assert a != b and a != c


def test_bucket_uniform_and_sign_balanced():
    n, r = 200000, 64
    bucket, sign = streams.bucket_sign(2024, r, np.arange(n))
    assert bucket.min() >= 0 and bucket.max() < r
    counts = np.bincount(bucket, minlength=r)
    chi2 = ((counts - n / r) ** 2 / (n / r)).sum()
    assert stats.chi2.sf(chi2, r - 1) > 1e-4
    assert set(np.unique(sign)) == {-1, 1}
    assert abs(sign.sum()) < 5 * np.sqrt(n)


def test_gaussian_moments_and_ks():
    a = np.arange(50000)[:, None]
    b = np.arange(4)[None, :]
    z = streams.gaussian(7, streams.STREAM_GAUSS_S, a, b).ravel()
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # the two Box-Muller outputs of one block are independent
    assert abs(np.corrcoef(z[0::2], z[1::2])[0, 1]) < 5 / np.sqrt(z.size / 2)


def test_gaussian_is_counter_based():
    full = streams.gaussian(9, 4, np.arange(10)[:, None], np.arange(6)[None, :])
    one = streams.gaussian(9, 4, np.array([7]), np.array([3]))
    assert full[7, 3] == one[0]


def test_pi2_scale():
    p = streams.pi2_matrix(3, 400, 64)
    assert p.shape == (400, 64)
    # column norms^2 ~ d/k
    assert abs((p * p).sum(0).mean() - 400 / 64) < 0.5


def test_gaussian_f32_matches_exact_box_muller():
    """The FP32 generator equals the Box-Muller transform of the same two
    24-bit uniforms (computed in FP64 with libm) to FP32 accuracy."""
    i = np.arange(4000, dtype=np.uint64)
    j = np.full(4000, 7, dtype=np.uint64)
    g = i >> np.uint64(2)
    w = streams.philox4x32_10(g, np.zeros_like(g), j, np.full(4000, 3, np.uint64), 11, 0)
    r = (i & np.uint64(3)).astype(int)
    wa = np.where(r < 2, w[0], w[2])
    wb = np.where(r < 2, w[1], w[3])
    u1 = ((wa >> np.uint64(8)).astype(np.float64) + 1.0) * 2.0 ** -24
    u2 = (wb >> np.uint64(8)).astype(np.float64) * 2.0 ** -24
    rad = np.sqrt(-2.0 * np.log(u1))
    ex = np.where(r % 2 == 0, rad * np.cos(2 * np.pi * u2), rad * np.sin(2 * np.pi * u2))
    got = streams.gaussian_f32(11, 3, i, j).astype(np.float64)
    assert np.max(np.abs(got - ex)) < 4e-6


def test_gaussian_f32_distribution():
    z = streams.gaussian_f32(5, 3, np.arange(100000)[:, None],
                             np.arange(4)[None, :]).ravel().astype(np.float64)
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1) < 6 * np.sqrt(2 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4


def test_bf16_round_ties_to_even():
    x = np.array([1.0, 1.00390625, 1.01171875, -3.3, 0.0], np.float32)
    want = np.array([1.0, 1.0, 1.015625, -3.296875, 0.0], np.float32)
    assert np.array_equal(streams.bf16_round(x), want)
