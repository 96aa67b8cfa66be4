"""Pins for the oracle's ordering and metrics, and the input generators."""
import numpy as np
import pytest

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


# ---- sampling policies (Algorithm 4 steps 3-4) ---------------------------------
from scipy import stats  # noqa: E402
from oracle import streams  # noqa: E402


def _chi2_ok(counts, expected):
    keep = expected > 0
    chi2 = float(np.sum((counts[keep] - expected[keep]) ** 2 / expected[keep]))
    return stats.chi2.sf(chi2, int(keep.sum()) - 1) > 1e-4


def test_swr_frequencies_follow_p():
    s = np.tile(np.array([1.0, 2.0, 3.0, 4.0], np.float32), 50)   # n = 200
    counts = np.zeros(s.shape[0])
    for ep in range(40):
        counts += np.bincount(order.swr_order(s, 7, ep), minlength=s.shape[0])
    p = s / s.sum()
    assert _chi2_ok(counts, p * counts.sum())


def test_swr_never_draws_zero_probability_rows():
    # w = [1, 0, 1, ...]: a draw landing on a cumulative boundary must not
    # pick the zero-weight row after it
    s = np.array([1.0, 0.0, 1.0, 0.0, -3.0, np.nan, 2.0, 0.0], np.float32)
    for ep in range(200):
        d = order.swr_order(s, 3, ep)
        assert set(d.tolist()) <= {0, 2, 6}
    one = np.zeros(50, np.float32)
    one[17] = 0.25
    assert np.all(order.swr_order(one, 1, 0) == 17)


def test_swr_rejects_no_positive_score():
    with pytest.raises(ValueError):
        order.swr_order(np.zeros(5, np.float32), 1, 0)


def test_swor_is_a_permutation_with_zero_scores_last():
    s = np.random.default_rng(2).random(300).astype(np.float32)
    s[[5, 40, 41, 299]] = 0.0
    p = order.swor_order(s, 11, 4)
    assert sorted(p.tolist()) == list(range(300))
    assert p[-4:].tolist() == [5, 40, 41, 299]


def test_swor_first_and_second_positions_follow_sequential_sampling():
    """Without-replacement draws: P(first = i) = P_i and
    P(second = j) = sum_{i != j} P_i P_j / (1 - P_i)."""
    s = np.array([1.0, 2.0, 5.0], np.float32)
    p = s / s.sum()
    first, second = np.zeros(3), np.zeros(3)
    epochs = 3000
    for ep in range(epochs):
        o = order.swor_order(s, 5, ep)
        first[o[0]] += 1
        second[o[1]] += 1
    assert _chi2_ok(first, p * epochs)
    p2 = np.array([sum(p[i] * p[j] / (1 - p[i]) for i in range(3) if i != j)
                   for j in range(3)])
    assert _chi2_ok(second, p2 * epochs)


def test_swor_exponentials_are_exponential():
    w0, _ = streams.sample_words(9, streams.STREAM_SWOR, 0, np.arange(20000))
    e = -streams.ln_f32(streams.unit_f32(w0)).astype(np.float64)
    assert stats.kstest(e, "expon").pvalue > 1e-4
    # the FP32 logarithm against libm on the same units
    u = streams.unit_f32(w0).astype(np.float64)
    assert np.max(np.abs(-np.log(u) - e)) < 2e-6


def test_swor_equal_scores_uniform_first():
    s = np.ones(8, np.float32)
    first = np.zeros(8)
    for ep in range(1600):
        first[order.swor_order(s, 13, ep)[0]] += 1
    assert _chi2_ok(first, np.full(8, 200.0))
