"""Pins for the oracle's exact and sketched leverage scores (CPU only).

Exact scores are pinned to the hat-matrix definition (pseudo-inverse brute
force), closed forms and invariants; sketched scores to the deterministic
subspace-embedding bound realised by the drawn sketch (Definition 1 and
Theorem 1), to the SVD form of Algorithm 2, and to the chi-square law of the
second projection.
"""
import math

import numpy as np
import pytest
from scipy import stats

import synth
from oracle import leverage as lv
from oracle import sketch as sk
from oracle import streams


def _hat_diag(x):
    """Brute force: diag(X X^+) with numpy's pseudo-inverse."""
    return np.einsum("ij,ji->i", x, np.linalg.pinv(x))


@pytest.mark.parametrize("n,d", [(12, 3), (40, 7), (64, 16)])
def test_exact_matches_pinv_bruteforce(n, d):
    x = np.random.default_rng(n).standard_normal((n, d)) * \
        np.exp(np.random.default_rng(d).standard_normal(n))[:, None]
    lev, rank = lv.exact_leverage(x)
    assert rank == d
    np.testing.assert_allclose(lev, _hat_diag(x), rtol=1e-10, atol=1e-14)


def test_exact_invariants_and_rank_deficient_bruteforce():
    rng = np.random.default_rng(2)
    n, d, k = 60, 10, 4
    x = rng.standard_normal((n, k)) @ rng.standard_normal((k, d))
    lev, rank = lv.exact_leverage(x)
    assert rank == k
    assert abs(lev.sum() - k) < 1e-10
    assert lev.min() >= -1e-15 and lev.max() <= 1 + 1e-12
    np.testing.assert_allclose(lev, _hat_diag(x), rtol=1e-8, atol=1e-12)


def test_closed_forms():
    rng = np.random.default_rng(3)
    # orthonormal columns: l_i = ||x_i||^2
    q = synth.haar(rng, 200, 6)
    lev, _ = lv.exact_leverage(q)
    np.testing.assert_allclose(lev, (q * q).sum(1), rtol=1e-11, atol=1e-15)
    # rank one: l_i = u_i^2 / ||u||^2
    u = rng.standard_normal(50)
    lev, rank = lv.exact_leverage(np.outer(u, [1.0, -2.0, 0.5]))
    assert rank == 1
    np.testing.assert_allclose(lev, u * u / (u @ u), rtol=1e-10)
    # [I_d; 0]: ones on the first d rows, zeros below
    x = np.vstack([np.eye(5), np.zeros((20, 5))])
    lev, _ = lv.exact_leverage(x)
    np.testing.assert_allclose(lev[:5], 1.0, rtol=1e-14)
    assert np.all(lev[5:] == 0.0)


def test_zero_row_scores_zero_and_equivariance():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((80, 6))
    x[17] = 0.0
    lev, _ = lv.exact_leverage(x)
    assert lev[17] == 0.0
    # X -> X T (invertible T) leaves the scores unchanged
    t = rng.standard_normal((6, 6)) + 3 * np.eye(6)
    lev2, _ = lv.exact_leverage(x @ t)
    np.testing.assert_allclose(lev2, lev, rtol=1e-9, atol=1e-15)
    # a row permutation permutes the scores
    p = rng.permutation(80)
    lev3, _ = lv.exact_leverage(x[p])
    np.testing.assert_allclose(lev3, lev[p], rtol=1e-10, atol=1e-15)


def _alg2_svd_form(x, sx):
    """Algorithm 2 as printed (SVD of SA, then A V Sigma^-1), for comparison."""
    _, s, vt = np.linalg.svd(sx, full_matrices=False)
    ua = (x @ vt.T) / s[None, :]
    return (ua * ua).sum(1)


def test_qr_form_equals_svd_form_of_algorithm2():
    x = synth.config0(n=3000, d=16, seed=11)
    out = lv.sketched_leverage(x, seed=5, r=512, k=0)
    ref = _alg2_svd_form(x, out["SX"])
    np.testing.assert_allclose(out["scores"], ref, rtol=1e-11)


def test_sketched_scores_within_realised_embedding_bound():
    """Def. 1 / Thm. 1: with X = U T (U orthonormal), the sketched score of
    every row lies in [l_i / sigma_max(SU)^2, l_i / sigma_min(SU)^2]."""
    x = synth.config0(n=5000, d=12, seed=12)
    lev, _ = lv.exact_leverage(x)
    q, _ = np.linalg.qr(x)
    out = lv.sketched_leverage(x, seed=9, r=1024, k=0)
    sq = sk.countsketch_dense(q, 9, 1024)
    sv = np.linalg.svd(sq, compute_uv=False)
    ratio = out["scores"] / lev
    assert ratio.min() >= (1 - 1e-9) / sv[0] ** 2
    assert ratio.max() <= (1 + 1e-9) / sv[-1] ** 2
    eps_hat = max(sv[0] ** 2 - 1, 1 - sv[-1] ** 2)
    assert eps_hat < 0.5


def test_osnap_scores_within_realised_embedding_bound():
    """The same bound with the OSNAP sketch (s = 2 nonzeros per column)."""
    x = synth.config0(n=5000, d=12, seed=14)
    lev, _ = lv.exact_leverage(x)
    q, _ = np.linalg.qr(x)
    out = lv.sketched_leverage(x, seed=10, r=512, k=0, kind="osnap", nnz=2)
    sq = sk.osnap_dense(q, 10, 512, 2)
    sv = np.linalg.svd(sq, compute_uv=False)
    ratio = out["scores"] / lev
    assert ratio.min() >= (1 - 1e-9) / sv[0] ** 2
    assert ratio.max() <= (1 + 1e-9) / sv[-1] ** 2
    assert max(sv[0] ** 2 - 1, 1 - sv[-1] ** 2) < 0.5


def test_injective_sketch_gives_exact_scores():
    n, d, r = 60, 5, 1 << 16
    for seed in range(100):
        b, _ = streams.bucket_sign(seed, r, np.arange(n))
        if len(set(b.tolist())) == n:
            break
    x = np.random.default_rng(6).standard_normal((n, d))
    out = lv.sketched_leverage(x, seed=seed, r=r, k=0)
    lev, _ = lv.exact_leverage(x)
    np.testing.assert_allclose(out["scores"], lev, rtol=1e-11)


def test_k0_is_no_projection():
    x = synth.config0(n=2000, d=10, seed=13)
    out = lv.sketched_leverage(x, seed=3, r=256, k=0)
    rinv = np.linalg.inv(lv.qr_r(out["SX"]))
    y = x @ rinv
    np.testing.assert_allclose(out["scores"], (y * y).sum(1), rtol=1e-10)


def test_pi2_ratio_is_chi2_over_k():
    """For a fixed row, l_hat / l_tilde ~ chi2_k / k over Pi_2 draws."""
    x = synth.config0(n=400, d=8, seed=14)
    sx = sk.countsketch_dense(x, 1, 128)
    base = lv.sketched_leverage(x, seed=1, r=128, k=0, sx=sx)["scores"]
    k = 16
    ratios = []
    for seed in range(300):
        s = lv.sketched_leverage(x, seed=seed, r=128, k=k, sx=sx)["scores"]
        ratios.append(s[0] / base[0])
    p = stats.kstest(np.array(ratios) * k, stats.chi2(k).cdf).pvalue
    assert p > 1e-3


def test_refined_equals_exact():
    x = synth.config0(n=3000, d=16, seed=15)
    out = lv.sketched_leverage(x, seed=2, r=256, k=0, refine=True)
    lev, _ = lv.exact_leverage(x)
    np.testing.assert_allclose(out["scores"], lev, rtol=1e-10)


def test_rank_deficient_truncation_restores_bound():
    """Figs. 2-3 analog: noise-free rank d/2 input. Without truncation
    (tau = 0) the scores are far off or non-finite; with the default tau the
    rank is found and the scores obey the embedding bound against the exact
    rank-d/2 leverage."""
    rng = np.random.default_rng(16)
    n, d, k = 4000, 16, 8
    u = synth.haar(rng, n, k)
    x = (u * np.exp(rng.standard_normal(n))[:, None]) @ rng.standard_normal((k, d))
    lev, rank = lv.exact_leverage(x)
    assert rank == k
    bad = lv.sketched_leverage(x, seed=4, r=1024, k=0, rank_tol=0.0)["scores"]
    assert (not np.all(np.isfinite(bad))) or \
        np.max(np.abs(bad - lev) / np.maximum(lev, 1e-300)) > 1.0
    good = lv.sketched_leverage(x, seed=4, r=1024, k=0)
    assert good["rank"] == k
    q, _ = np.linalg.qr(x)
    sq = sk.countsketch_dense(q, 4, 1024)
    # basis of the column space: the first k left singular vectors of X
    ux = np.linalg.svd(x, full_matrices=False)[0][:, :k]
    sv = np.linalg.svd(sk.countsketch_dense(ux, 4, 1024), compute_uv=False)
    ratio = good["scores"] / lev
    assert ratio.min() >= (1 - 1e-6) / sv[0] ** 2
    assert ratio.max() <= (1 + 1e-6) / sv[-1] ** 2


def test_small_singular_values_truncated_by_threshold():
    """Fig. 5 analog: exact low rank plus tiny noise looks full rank; a rank
    tolerance above the noise level truncates it, one below keeps it."""
    rng = np.random.default_rng(17)
    n, d, k = 3000, 12, 6
    x = synth.haar(rng, n, k) @ rng.standard_normal((k, d))
    x += 1e-9 * rng.standard_normal((n, d))
    lo = lv.sketched_leverage(x, seed=1, r=512, k=0, rank_tol=1e-14)
    hi = lv.sketched_leverage(x, seed=1, r=512, k=0, rank_tol=1e-6)
    assert lo["rank"] == d
    assert hi["rank"] == k
    assert abs(hi["scores"].sum() - k) < 0.5


def test_sketched_svd_matches_r_factor_and_gram():
    """Sigma of S X equals sigma of its QR factor R (Q is orthonormal), and
    V Sigma^2 V^T is the Gram matrix (S X)^T (S X)."""
    x = synth.config0(n=3000, d=20, seed=15)
    sig, v = lv.sketched_svd(x, 4, 256)
    sx = sk.countsketch_dense(x, 4, 256)
    np.testing.assert_allclose(sig, np.linalg.svd(lv.qr_r(sx), compute_uv=False),
                               rtol=1e-12)
    np.testing.assert_allclose(v @ np.diag(sig ** 2) @ v.T, sx.T @ sx,
                               rtol=1e-10, atol=1e-10 * sig[0] ** 2)
    np.testing.assert_allclose(v.T @ v, np.eye(20), atol=1e-13)
    assert np.all(np.diff(sig) <= 0)
    assert np.all(v[np.argmax(np.abs(v), axis=0), np.arange(20)] > 0)


def test_always_svd_rank_catches_kahan_matrix():
    """A Kahan-type R has a benign diagonal but a tiny singular value: the
    diagonal screen calls it full rank, the SVD decision does not."""
    d, c = 60, 0.3
    s_ = math.sqrt(1 - c * c)
    kahan = np.triu(-c * np.ones((d, d)), 1) + np.eye(d)
    kahan = np.diag(s_ ** np.arange(d)) @ kahan
    sv = np.linalg.svd(kahan, compute_uv=False)
    tol = (sv[-1] / sv[0]) * 10.0          # the smallest value falls below it
    rank, full, dmin, dmax, _ = lv.rank_decision(kahan, tol)
    assert full and rank == d               # the screen misses it
    assert dmin > math.sqrt(tol) * dmax
    rank2, full2, _, _, _ = lv.rank_decision(kahan, tol, always_svd=True)
    assert not full2 and rank2 == d - 1


# ---- realised distortion (Def. 1 / Thm. 1) -------------------------------------
def test_realised_distortion_zero_for_injective_sketch():
    """An injective CountSketch maps U to a signed row permutation of U:
    S U has orthonormal columns, eps_hat = 0 (to rounding)."""
    n, d, r = 60, 5, 1 << 16
    for seed in range(100):
        b, _ = streams.bucket_sign(seed, r, np.arange(n))
        if len(set(b.tolist())) == n:
            break
    x = np.random.default_rng(6).standard_normal((n, d))
    assert lv.realised_distortion(x, seed, r) < 1e-13


def test_realised_distortion_brackets_the_scores():
    """Thm. 1 with Def. 1: every sketched score (k = 0) lies in
    [l_i / (1 + eps_hat), l_i / (1 - eps_hat)]."""
    x = synth.config0(n=4000, d=10, seed=31)
    eps = lv.realised_distortion(x, 7, 512)
    lev, _ = lv.exact_leverage(x)
    got = lv.sketched_leverage(x, seed=7, r=512, k=0)["scores"]
    ratio = got / lev
    assert 0.0 < eps < 1.0
    assert ratio.min() >= (1 - 1e-9) / (1 + eps)
    assert ratio.max() <= (1 + 1e-9) / (1 - eps)


def test_realised_distortion_gaussian_matches_marchenko_pastur():
    """FP64 Gaussian S (N(0, 1/r) entries) on a d-dimensional subspace: the
    squared singular values of S U fill [(1 - sqrt(d/r))^2, (1 + sqrt(d/r))^2]
    as r grows, so eps_hat ~ 2 sqrt(d/r) + d/r; checked within 25 % over
    four seeds at d = 20, r = 2000."""
    x = np.random.default_rng(3).standard_normal((3000, 20))
    edge = 2 * np.sqrt(20 / 2000) + 20 / 2000
    vals = [lv.realised_distortion(x, s, 2000, kind="gaussian",
                                   precision="f64") for s in range(4)]
    assert 0.75 * edge < np.mean(vals) < 1.25 * edge


def test_realised_distortion_equals_sketch_r_over_exact_r():
    """sigma(S U) = sigma(R_S R^-1) with R_S the R of S X D and R the R of
    X D (S X D = Q_S R_S and X D = Q R give S Q = Q_S R_S R^-1): the route a
    factor-only implementation takes."""
    x = synth.config0(n=3000, d=16, seed=33)
    out = lv.sketched_leverage(x, seed=5, r=256, k=0)
    rd = lv.qr_r(x * out["D"][None, :])
    sv = np.linalg.svd(out["R_D"] @ np.linalg.inv(rd), compute_uv=False)
    eps = max(sv[0] ** 2 - 1, 1 - sv[-1] ** 2)
    assert abs(eps - lv.realised_distortion(x, 5, 256)) < 1e-12
