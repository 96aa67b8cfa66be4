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


# ---- quantile form of the sketch entries (BF16 / FP8 inputs) ----------------
def test_half_normal_quantiles_against_library_halfnorm():
    """t_m against scipy's half-normal quantile function (a separate routine
    from erfinv), and the first cells against erfinv's leading term
    sqrt(pi)/2 p: t_m ~ sqrt(pi/2) (2m + 1) / 65536."""
    t = streams.half_normal_quantiles()
    m = np.arange(streams.QCELLS)
    assert np.all(np.diff(t) > 0)
    ref = stats.halfnorm.ppf((m + 0.5) / streams.QCELLS)
    assert np.max(np.abs(t - ref) / t) < 1e-12
    lead = np.sqrt(np.pi / 2) * (2 * m[:4] + 1) / 65536.0
    assert np.max(np.abs(t[:4] - lead) / lead) < 1e-8


def _rounding_margin(t, fmt):
    """Relative distance of each t to the nearest rounding boundary (midpoint
    of two neighbours) of the format."""
    _, ex = np.frexp(t)
    e = ex - 1
    sp = np.ldexp(1.0, e - 7) if fmt == "bf16" else \
        np.ldexp(1.0, np.maximum(e, -6) - 3)
    fr = t / sp - np.floor(t / sp)
    return np.abs(fr - 0.5) * sp / t


def test_quantile_tables_well_defined_and_rounded():
    """No t_m lies within 1e-9 (relative) of a rounding boundary, so the
    tables do not depend on how erfinv is evaluated; the roundings agree with
    independent implementations: torch's FP64 -> bfloat16 conversion, and the
    e4m3 quantiser of the input generators (nearest representable value by
    search, a column with maximum 448 so that its scale is 1)."""
    import synth
    torch = pytest.importorskip("torch")
    t = streams.half_normal_quantiles()
    for fmt in ("bf16", "fp8"):
        assert _rounding_margin(t, fmt).min() > 1e-9
    tb = streams.quantile_table("bf16")
    assert np.array_equal(
        tb, torch.from_numpy(t).to(torch.bfloat16).to(torch.float64).numpy())
    codes, cs = synth.to_fp8_e4m3(np.concatenate([t, [448.0]])[:, None])
    assert cs[0] == 1.0
    t8 = streams.quantile_table("fp8")
    assert np.array_equal(t8, synth.fp8_e4m3_to_f64(codes, cs)[:-1, 0])
    # e4m3: the cells below 2^-10 round to zero, the largest to 4.5
    assert t8[0] == 0.0 and t8[-1] == 4.5
    # rounding ties go to the even neighbour
    assert np.array_equal(streams.round_to_format(
        np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 0.0]), "bf16"),
        [1.0, 1.0 + 2.0 ** -6, 0.0])
    assert np.array_equal(streams.round_to_format(
        np.array([1.0625, 1.1875, 2.0 ** -10, 3 * 2.0 ** -10, 500.0]), "fp8"),
        [1.0, 1.25, 0.0, 2.0 ** -8, 448.0])


def test_gaussian_q_block_layout_and_counter():
    """Entry (i, j) from its own Philox block equals the block-split matrix
    at any row offset; the eight data rows of one block are its eight 16-bit
    halves, low half first, words in order."""
    j = np.arange(37)[:, None]
    for row0, n in ((0, 64), (5, 1001), (2 ** 33 + 3, 29)):
        i = np.arange(row0, row0 + n, dtype=np.uint64)[None, :]
        for fmt in ("bf16", "fp8"):
            a = streams.gaussian_q(11, i, j, fmt)
            b = streams.gaussian_sketch_matrix_q(11, 37, n, fmt, row0=row0)
            assert np.array_equal(a, b)
    w = streams.philox4x32_10(np.uint64(3), np.uint64(0), np.uint64(5),
                              np.uint64(streams.STREAM_GAUSS_Q), 77, 0)
    halves = [int(x) & 0xFFFF if h == 0 else int(x) >> 16
              for x in w for h in (0, 1)]
    got = streams.gaussian_q_halfwords(77, np.arange(24, 32), 5)
    assert list(got) == halves


def test_gaussian_q_distribution():
    """Sample of 400000 entries: halves uniform over 2^16 values (chi^2 on
    256 bins of the top byte and on the low byte), signs balanced, mean 0,
    variance that of the table, neighbouring entries uncorrelated. The law
    of a BF16 entry (2^16 equiprobable signed cells) is within 2^-9 of
    N(0,1) in Kolmogorov distance (BF16 rounding moves a quantile z by at
    most 2^-8 |z|, and z phi(z) <= 0.25), and the sample's KS statistic
    within that plus sampling noise."""
    i = np.arange(100000)[None, :]
    j = np.arange(4)[:, None]
    v = streams.gaussian_q_halfwords(2024, i, j).ravel()
    for byte in (v >> 8, v & 0xFF):
        c = np.bincount(byte, minlength=256)
        chi2 = ((c - v.size / 256) ** 2 / (v.size / 256)).sum()
        assert stats.chi2.sf(chi2, 255) > 1e-4
    for fmt in ("bf16", "fp8"):
        z = streams.gaussian_sketch_matrix_q(2024, 4, 100000, fmt).ravel()
        tab = streams.quantile_table(fmt)
        assert abs(z.mean()) < 5 / np.sqrt(z.size)
        assert abs(z.var() - (tab ** 2).mean()) < 6 * np.sqrt(2 / z.size)
        assert abs((tab ** 2).mean() - 1) < (2e-5 if fmt == "bf16" else 1e-3)
        if fmt == "bf16":
            # exact Kolmogorov distance of the table's law: the CDF jumps by
            # 2^-16 at each signed value; compare both sides of every jump
            vals = np.sort(np.concatenate([-tab, tab]))
            cdf_hi = np.arange(1, vals.size + 1) / vals.size
            phi = stats.norm.cdf(vals)
            law_ks = max(np.abs(cdf_hi - phi).max(),
                         np.abs(cdf_hi - 2.0 ** -16 - phi).max())
            assert law_ks < 2.0 ** -9
            ks = stats.kstest(z, "norm").statistic
            assert ks < law_ks + 1.63 / np.sqrt(z.size)
        assert abs(np.corrcoef(z[:-1], z[1:])[0, 1]) < 5 / np.sqrt(z.size)
