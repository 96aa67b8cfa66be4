"""Leverage scores: exact (Sec. 2.2, Algorithm 1) and sketched (Algorithms 2, 3).

Definitions followed (Sec. 2.2): the leverage of row i is the i-th diagonal
entry of the hat matrix H = A (A^T A)^+ A^T, which equals ||U_i||^2 for the
thin SVD A = U Sigma V^T, and equally ||Q_i||^2 for a thin QR A = Q R of a
full-column-rank A.

Algorithm 2 in QR form: with SA = Q R, R^{-1} = V Sigma^{-1} (U^T Q) where
SA = U Sigma V^T, and U^T Q is orthogonal, so ||a_i R^{-1}|| = ||a_i V
Sigma^{-1}|| (the printed A V^T Sigma^{-1} of Algorithm 2 step 3 is read as
A V Sigma^{-1}, the dimensionally consistent form).

Numerical rank (Sec. 3.3-3.5, Algorithm 3): the threshold of Algorithm 3 is
read as *relative*, tau (default 1e-10), applied to the R of the equilibrated
sketch R_D. A cheap screen on diag(R_D) decides first: if min |r_jj| >
sqrt(tau) max |r_jj| the factor is taken as full rank; otherwise the rank and
the truncated basis come from the SVD of R_D (Algorithm 3 step 3, since the
singular values of R equal those of SA): rank = #{sigma_j > tau sigma_1}.

The truncated inverse is the pseudo-inverse of the rank-r truncation of R_D,
V' Sigma'^{-1} U'^T. Its row norms after X are those of Algorithm 3 step 4
(U'^T has orthonormal rows), and it equals R_D^{-1} when nothing is truncated.

Second projection: M = D pinv_r(R_D) Pi_2 with Pi_2 (d x k) N(0, 1/k) entries
(the fast leverage estimator of Drineas et al., cited in Sec. 2.2 and 3),
k = 0 meaning Pi_2 = I. Scores: l_i = ||x_i M||^2.

R is normalised to a non-negative diagonal (the unique QR factor of a
full-rank matrix), so that R^{-1} Pi_2 does not depend on the sign choices of
a particular QR routine.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import sketch as sk
from . import streams

DEFAULT_RANK_TOL = 1e-10


def positive_r(r: np.ndarray) -> np.ndarray:
    """Flip row signs of an upper-triangular R so its diagonal is >= 0."""
    s = np.sign(np.diag(r)).copy()
    s[s == 0] = 1.0
    return r * s[:, None]


def qr_r(a: np.ndarray) -> np.ndarray:
    """R factor (d x d, non-negative diagonal) of a Householder QR of a (m >= d)."""
    r = np.linalg.qr(np.asarray(a, dtype=np.float64), mode="r")
    return positive_r(r)


def rank_decision(r: np.ndarray, rank_tol: float = DEFAULT_RANK_TOL,
                  always_svd: bool = False):
    """Numerical rank of an upper-triangular R (Algorithm 3 step 3).

    Returns (rank, screened_full, diag_min, diag_max, svd) where svd is
    (U, sigma, Vt) when the diagonal screen tripped (or ``always_svd``: the
    rank is always decided by the singular values, which a diagonal screen
    can misjudge on Kahan-type R), else None.
    """
    dg = np.abs(np.diag(r))
    dmin, dmax = float(dg.min()), float(dg.max())
    d = r.shape[0]
    if not always_svd and dmax > 0.0 and dmin > math.sqrt(rank_tol) * dmax:
        return d, True, dmin, dmax, None
    u, s, vt = np.linalg.svd(r)
    if s[0] == 0.0:
        rank = 0
    else:
        rank = int(np.count_nonzero(s > rank_tol * s[0]))
    return rank, False, dmin, dmax, (u, s, vt)


def truncated_apply(r: np.ndarray, rhs: np.ndarray,
                    rank_tol: float = DEFAULT_RANK_TOL,
                    always_svd: bool = False):
    """pinv_rank(R) @ rhs, with the rank from ``rank_decision``.

    Full rank: a triangular solve R M = rhs. Otherwise V' Sigma'^-1 U'^T rhs.
    Returns (M, rank, info-dict).
    """
    rank, full, dmin, dmax, svd = rank_decision(r, rank_tol, always_svd)
    info = {"rank": rank, "screen_full": full, "diag_min": dmin,
            "diag_max": dmax}
    if full:
        m = sla.solve_triangular(r, rhs, lower=False)
    else:
        u, s, vt = svd
        ut = u[:, :rank].T @ rhs
        m = vt[:rank].T @ (ut / s[:rank, None])
    return m, rank, info


def row_scores(x, m: np.ndarray) -> np.ndarray:
    """l_i = ||x_i M||^2 (FP64)."""
    if isinstance(x, np.ndarray):
        y = np.asarray(x, dtype=np.float64) @ m
    else:
        y = _csr(x) @ m
    return np.einsum("ij,ij->i", y, y)


def _csr(csr):
    return sp.csr_matrix((csr.val.astype(np.float64), csr.col_idx,
                          csr.row_ptr), shape=(csr.n, csr.d))


def _colmax(x):
    if isinstance(x, np.ndarray):
        return sk.colmax_dense(x)
    return sk.colmax_csr(x)


def exact_leverage(x: np.ndarray, rank_tol: float = DEFAULT_RANK_TOL):
    """Exact scores diag(X X^+) of the rank-truncated X (Algorithm 1, QR form).

    Returns (scores, rank).
    """
    xf = np.asarray(x, dtype=np.float64)
    dsc = sk.column_scale(sk.colmax_dense(xf))
    q, r = np.linalg.qr(xf * dsc[None, :])
    sgn = np.sign(np.diag(r)).copy()
    sgn[sgn == 0] = 1.0
    q = q * sgn[None, :]
    r = r * sgn[:, None]
    rank, full, _, _, svd = rank_decision(r, rank_tol)
    if full:
        return np.einsum("ij,ij->i", q, q), rank
    u = svd[0]
    qu = q @ u[:, :rank]
    return np.einsum("ij,ij->i", qu, qu), rank


def sketch_of(x, seed: int, r: int, kind: str = "countsketch",
              precision: str = "bf16", nnz: int = 2) -> np.ndarray:
    """Unscaled sketch S X (FP64). For the Gaussian sketch, ``precision``
    names the entries of S ("bf16" / "fp8": the quantile form for BF16 / FP8
    inputs, "f32": the plain FP32 path, "f64": the FP64 stream); for OSNAP,
    ``nnz`` is the
    number of nonzeros per column of S."""
    if kind == "countsketch":
        if isinstance(x, np.ndarray):
            return sk.countsketch_dense(x, seed, r)
        return sk.countsketch_csr(x, seed, r)
    if kind == "osnap":
        if isinstance(x, np.ndarray):
            return sk.osnap_dense(x, seed, r, nnz)
        return sk.osnap_csr(x, seed, r, nnz)
    if kind == "srht":
        if not isinstance(x, np.ndarray):
            x = x.to_dense()
        return sk.srht_dense(x, seed, r)
    if kind == "gaussian":
        if not isinstance(x, np.ndarray):
            x = x.to_dense()
        return sk.gaussian_sketch_dense(x, seed, r, precision=precision)
    raise ValueError(kind)


def sketched_svd(x, seed: int, r: int, kind: str = "countsketch",
                 precision: str = "bf16", nnz: int = 2):
    """Sketched SVD S X = U Sigma V^T (Algorithm 2 step 2): sigma
    (descending) and V (d x d, column j the right singular vector of
    sigma_j, its largest-magnitude entry made positive; the first such entry
    when several tie)."""
    sx = sketch_of(x, seed, r, kind, precision, nnz)
    _, sig, vt = np.linalg.svd(sx, full_matrices=False)
    v = vt.T.copy()
    for j in range(v.shape[1]):
        i = int(np.argmax(np.abs(v[:, j])))
        if v[i, j] < 0:
            v[:, j] = -v[:, j]
    return sig, v


def sketched_leverage(x, seed: int, r: int, k: int, kind: str = "countsketch",
                      rank_tol: float = DEFAULT_RANK_TOL, sx=None,
                      refine: bool = False, precision: str = "bf16",
                      nnz: int = 2, always_svd: bool = False):
    """Algorithm 3 in QR form with the second projection Pi_2.

    ``sx`` may carry a precomputed unscaled sketch. With ``refine`` the factor
    is the exact R of X D (the fixed point of the sketch-preconditioned
    Cholesky-QR refinement, independent of S).
    Returns a dict with scores, rank, R_D, D, M, SX.
    """
    d = x.shape[1] if isinstance(x, np.ndarray) else x.d
    dsc = sk.column_scale(_colmax(x))
    if refine:
        xd = (x.to_dense() if not isinstance(x, np.ndarray)
              else np.asarray(x, dtype=np.float64)) * dsc[None, :]
        rd = qr_r(xd)
    else:
        if sx is None:
            sx = sketch_of(x, seed, r, kind, precision, nnz)
        rd = qr_r(sx * dsc[None, :])
    pi = np.eye(d) if k == 0 else streams.pi2_matrix(seed, d, k)
    mp, rank, info = truncated_apply(rd, pi, rank_tol, always_svd)
    m = dsc[:, None] * mp
    scores = row_scores(x, m)
    return {"scores": scores, "rank": rank, "R_D": rd, "D": dsc, "M": m,
            "SX": sx, "info": info}


def realised_distortion(x, seed: int, r: int, kind: str = "countsketch",
                        precision: str = "bf16", nnz: int = 2) -> float:
    """Realised distortion of the sketch on the column space of X (Def. 1 and
    Thm. 1, Sec. 2.1): with U an orthonormal basis of range(X) (the Q of a
    Householder QR of X D; X of full column rank),
        eps_hat = max(sigma_max(S U)^2 - 1, 1 - sigma_min(S U)^2),
    the smallest eps for which S is a (1 +- eps) subspace embedding of X,
    ||S X v||^2 in [(1 - eps), (1 + eps)] ||X v||^2 for every v. S is the
    sketch of ``sketch_of`` with the same seed (its entries do not depend on
    the matrix they multiply)."""
    xd = x.to_dense() if not isinstance(x, np.ndarray) else \
        np.asarray(x, dtype=np.float64)
    dsc = sk.column_scale(_colmax(x))
    q, _ = np.linalg.qr(xd * dsc[None, :])
    su = sketch_of(q, seed, r, kind, precision, nnz)
    sv = np.linalg.svd(su, compute_uv=False)
    return float(max(sv[0] ** 2 - 1.0, 1.0 - sv[-1] ** 2))
