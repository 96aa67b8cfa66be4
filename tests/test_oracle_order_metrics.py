"""Pins for the oracle's ordering and metrics, and the input generators."""
import numpy as np

import synth
from oracle import metrics, order


def test_dec_order_matches_library_stable_sort():
    rng = np.random.default_rng(0)
    s = rng.integers(0, 20, 500).astype(np.float32)   # many ties
    p = order.dec_order(s)
    assert np.array_equal(p, np.argsort(-s, kind="stable"))
    assert np.all(np.diff(s[p]) <= 0)


def test_dec_order_all_equal_is_identity():
    assert np.array_equal(order.dec_order(np.ones(37)), np.arange(37))


def test_kendall_tau_matches_bruteforce():
    rng = np.random.default_rng(1)
    a = rng.integers(0, 15, 300).astype(float)
    b = a + rng.integers(0, 5, 300)
    assert abs(metrics.kendall_tau(a, b) -
               metrics.kendall_tau_bruteforce(a, b)) < 1e-12


def test_max_rel_err():
    assert abs(metrics.max_rel_err([1.1, 0.0], [1.0, 0.0]) - 0.1) < 1e-12
    assert metrics.max_rel_err([1.0, 1e-30], [1.0, 0.0]) == float("inf")


def test_synth_shapes():
    x = synth.config0(n=500, d=16)
    assert x.shape == (500, 16) and x.dtype == np.float64
    y = synth.image_like(300, 64)
    assert y.dtype == np.float32 and y.min() >= 0 and y.max() <= 1
    c = synth.text_like_csr(3000, 512, seed=5)
    assert c.row_ptr[0] == 0 and c.row_ptr[-1] == c.col_idx.size
    assert np.all(np.diff(c.row_ptr) >= 1)
    for i in range(0, 3000, 97):
        cols = c.col_idx[c.row_ptr[i]:c.row_ptr[i + 1]]
        assert np.all(np.diff(cols) > 0)
    dens = c.nnz / (3000 * 512)
    assert 0.002 < dens < 0.01
    bits = synth.to_bf16_bits(np.array([1.0, -2.5, 1.00390625, 3.0e38]))
    back = synth.bf16_bits_to_f64(bits)
    assert back[0] == 1.0 and back[1] == -2.5 and back[2] == 1.0
