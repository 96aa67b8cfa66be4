"""Pins for the oracle's sketches and column equilibration (CPU only)."""
import math

import numpy as np
import pytest

import synth
from oracle import sketch as sk
from oracle import streams


def _explicit_countsketch(seed, r, n):
    """S as a dense r x n matrix, built entry by entry."""
    bucket, sign = streams.bucket_sign(seed, r, np.arange(n))
    s = np.zeros((r, n))
    for i in range(n):
        s[bucket[i], i] = sign[i]
    return s


def test_countsketch_equals_explicit_product():
    rng = np.random.default_rng(0)
    # small integers: every FP64 sum is exact, so the two orders agree exactly
    x = rng.integers(-50, 50, (300, 7)).astype(np.float64)
    s = _explicit_countsketch(11, 40, 300)
    assert np.array_equal(sk.countsketch_dense(x, 11, 40), s @ x)


def test_countsketch_ascending_order_fp64():
    # values whose FP64 sum depends on order: check the stated order
    x = np.array([[1e16], [1.0], [-1e16], [1.0]])
    bucket, sign = streams.bucket_sign(5, 1, np.arange(4))
    want = 0.0
    for i in range(4):
        want += sign[i] * x[i, 0]
    assert sk.countsketch_dense(x, 5, 1)[0, 0] == want


def test_injective_countsketch_is_signed_permutation():
    n, r = 50, 4096
    # find a seed whose bucket hash is collision-free on 50 rows
    for seed in range(100):
        b, s = streams.bucket_sign(seed, r, np.arange(n))
        if len(set(b.tolist())) == n:
            break
    x = np.random.default_rng(1).standard_normal((n, 5))
    sx = sk.countsketch_dense(x, seed, r)
    for i in range(n):
        assert np.array_equal(sx[b[i]], s[i] * x[i])


def test_csr_sketch_equals_dense_sketch():
    csr = synth.text_like_csr(2000, 300, density=0.02, seed=3)
    dense = csr.to_dense()
    a = sk.countsketch_csr(csr, 77, 128)
    b = sk.countsketch_dense(dense, 77, 128)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-12 * np.abs(b).max())


def test_gaussian_sketch_is_unbiased_embedding():
    # E[S^T S] = I for S = G / sqrt(r): average over many columns
    r, n = 4000, 6
    g = streams.gaussian_sketch_matrix(3, r, n)
    sts = (g.T @ g) / r
    assert np.abs(sts - np.eye(n)).max() < 6 / math.sqrt(r)
    x = np.eye(n)
    np.testing.assert_allclose(sk.gaussian_sketch_dense(x, 3, r), g / math.sqrt(r))


def test_column_scale_powers_of_two():
    cm = np.array([0.0, 1.0, 1.5, 2.0, 3.999, 1e-300, 7e200, 0.75])
    d = sk.column_scale(cm)
    assert d[0] == 1.0
    for m, s in zip(cm[1:], d[1:]):
        assert 1.0 <= m * s < 2.0
        mant, _ = math.frexp(s)
        assert mant == 0.5          # exact power of two


def test_scaled_sketch_is_exact():
    x = np.random.default_rng(4).standard_normal((500, 9)) * \
        np.array([1e-3, 1, 10, 1e5, 3, 0.1, 7, 2e-8, 1])
    dsc = sk.column_scale(sk.colmax_dense(x))
    a = sk.countsketch_dense(x * dsc, 8, 64)
    b = sk.countsketch_dense(x, 8, 64) * dsc
    assert np.array_equal(a, b)


# ---- OSNAP -------------------------------------------------------------------
def _explicit_osnap(seed, r, s, n):
    """S as a dense r x n matrix, built entry by entry from the hashes."""
    bucket, sign = streams.osnap_bucket_sign(seed, r, s, np.arange(n))
    m = np.zeros((r, n))
    for j in range(s):
        for i in range(n):
            m[bucket[j, i], i] += sign[j, i] / math.sqrt(s)
    return m


def test_osnap_with_one_nonzero_is_countsketch():
    x = synth.config0(n=700, d=9, seed=4)
    assert np.array_equal(sk.osnap_dense(x, 21, 96, 1),
                          sk.countsketch_dense(x, 21, 96))


def test_osnap_equals_explicit_product():
    rng = np.random.default_rng(1)
    # small integers and s = 4 (1/sqrt(s) = 0.5): every step is exact
    x = rng.integers(-50, 50, (300, 7)).astype(np.float64)
    assert np.array_equal(sk.osnap_dense(x, 13, 64, 4),
                          _explicit_osnap(13, 64, 4, 300) @ x)
    y = rng.standard_normal((257, 5))
    np.testing.assert_allclose(sk.osnap_dense(y, 14, 90, 3),
                               _explicit_osnap(14, 90, 3, 257) @ y,
                               rtol=1e-13, atol=1e-13)


def test_osnap_columns_have_one_entry_per_block():
    r, s, n = 120, 3, 400
    m = _explicit_osnap(7, r, s, n)
    b = r // s
    for i in range(n):
        nz = np.nonzero(m[:, i])[0]
        assert len(nz) == s
        assert sorted(nz // b) == list(range(s))
        np.testing.assert_allclose(np.abs(m[nz, i]), 1 / math.sqrt(s),
                                   rtol=1e-15)
        assert abs(np.dot(m[:, i], m[:, i]) - 1.0) < 1e-14


def test_osnap_is_unbiased_embedding():
    x = np.random.default_rng(3).standard_normal(64)
    vals = [np.sum(sk.osnap_dense(x[:, None], seed, 32, 2) ** 2)
            for seed in range(400)]
    # ||S x||^2 is unbiased for ||x||^2; 400 draws, 5 standard errors
    m, sd = np.mean(vals), np.std(vals) / math.sqrt(len(vals))
    assert abs(m - np.dot(x, x)) < 5 * sd


def test_osnap_csr_equals_dense():
    c = synth.text_like_csr(400, 60, seed=2)
    np.testing.assert_array_equal(sk.osnap_csr(c, 5, 48, 2),
                                  sk.osnap_dense(c.to_dense(), 5, 48, 2))


def test_osnap_rejects_s_not_dividing_r():
    with pytest.raises(ValueError):
        streams.osnap_bucket_sign(1, 10, 3, np.arange(5))


# ---- SRHT --------------------------------------------------------------------------
def test_srht_equals_explicit_product():
    """(1/sqrt(r)) P H D X against scipy's Hadamard matrix; integer X keeps
    every sum exact, so the two agree exactly."""
    import scipy.linalg
    rng = np.random.default_rng(4)
    x = rng.integers(-20, 20, (200, 6)).astype(np.float64)   # n' = 256
    n2, rows = sk.srht_plan(3, 200, 64)
    assert n2 == 256 and len(set(rows.tolist())) == 64
    h = scipy.linalg.hadamard(256)
    dx = np.zeros((256, 6))
    dx[:200] = sk.srht_signs(3, 200)[:, None] * x
    ref = (h @ dx)[rows] * (1.0 / math.sqrt(64))
    assert np.array_equal(sk.srht_dense(x, 3, 64), ref)


def test_srht_all_rows_is_orthogonal():
    """With r = n' the sketch is (1/sqrt(n')) H D times a permutation:
    orthogonal, so the Frobenius norm is kept."""
    x = np.random.default_rng(5).standard_normal((128, 9))
    sx = sk.srht_dense(x, 8, 128)
    np.testing.assert_allclose(np.linalg.norm(sx), np.linalg.norm(x), rtol=1e-13)
    np.testing.assert_allclose(sx.T @ sx, x.T @ x, rtol=1e-12, atol=1e-12)


def test_srht_is_unbiased_embedding():
    x = np.random.default_rng(6).standard_normal(100)
    vals = [np.sum(sk.srht_dense(x[:, None], seed, 16) ** 2) for seed in range(400)]
    m, sd = np.mean(vals), np.std(vals) / math.sqrt(len(vals))
    assert abs(m - np.dot(x, x)) < 5 * sd


def test_srht_rejects_r_above_padded_rows():
    with pytest.raises(ValueError):
        sk.srht_plan(1, 100, 200)


def test_colmax_csr_equals_colmax_of_dense():
    """Column max-abs of a CSR matrix equals that of its dense form (with
    negative values, empty columns and a column holding one entry)."""
    c = synth.text_like_csr(3000, 300, density=0.01, seed=21)
    c.val = (c.val * np.where(np.arange(c.nnz) % 3 == 0, -1.0, 1.0)).astype(
        np.float32)
    got = sk.colmax_csr(c)
    want = sk.colmax_dense(c.to_dense())
    assert np.array_equal(got, want)
    assert (want == 0).any()             # some column is empty
    # the equilibration derived from it is the same power of two
    assert np.array_equal(sk.column_scale(got), sk.column_scale(want))
