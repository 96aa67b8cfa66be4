"""Sketches S*X (Sec. 2.1; Algorithm 2 step 1), plain FP64 loops.

CountSketch follows the streaming model of Sec. 3.1.2: rows are read in
ascending order and row i is added, with sign s(i), into sketch row h(i). The
sums are FP64 and taken in ascending row order within each bucket.

The Gaussian sketch is S = G / sqrt(r) with G_{j,i} standard normal, so that
E[S^T S] = I (the scaling reading of the Gaussian family listed in Sec. 2.1).

Column equilibration: D_j = 2^-e_j with e_j = floor(log2 max_i |X_ij|)
(D_j = 1 for an all-zero column). Because D is a power of two,
S (X D) = (S X) D exactly, and leverage scores are invariant under X -> X D;
D only conditions the rank decision and the rounding.
"""
from __future__ import annotations

import math

import numpy as np

from . import streams


def column_scale(colmax: np.ndarray) -> np.ndarray:
    """Power-of-two column scales from column max-abs values."""
    out = np.ones(colmax.shape[0], dtype=np.float64)
    for j, m in enumerate(colmax):
        m = float(m)
        if m > 0.0 and math.isfinite(m):
            _, e = math.frexp(m)            # m = f * 2^e, f in [0.5, 1)
            out[j] = math.ldexp(1.0, -(e - 1))
    return out


def colmax_dense(x: np.ndarray) -> np.ndarray:
    return np.abs(np.asarray(x, dtype=np.float64)).max(axis=0)


def colmax_csr(csr) -> np.ndarray:
    out = np.zeros(csr.d, dtype=np.float64)
    np.maximum.at(out, csr.col_idx, np.abs(csr.val.astype(np.float64)))
    return out


def countsketch_dense(x: np.ndarray, seed: int, r: int,
                      row_offset: int = 0) -> np.ndarray:
    """SX (r x d, FP64): SX[h(i)] += s(i) x_i for i ascending."""
    n, d = x.shape
    bucket, sign = streams.bucket_sign(seed, r, np.arange(n) + row_offset)
    sx = np.zeros((r, d), dtype=np.float64)
    xf = np.asarray(x, dtype=np.float64)
    for i in range(n):
        sx[bucket[i]] += float(sign[i]) * xf[i]
    return sx


def countsketch_csr(csr, seed: int, r: int) -> np.ndarray:
    """CountSketch of a CSR matrix, same order as the dense form."""
    bucket, sign = streams.bucket_sign(seed, r, np.arange(csr.n))
    sx = np.zeros((r, csr.d), dtype=np.float64)
    rp = csr.row_ptr
    for i in range(csr.n):
        a, b = int(rp[i]), int(rp[i + 1])
        if b > a:
            sx[bucket[i], csr.col_idx[a:b]] += float(sign[i]) * \
                csr.val[a:b].astype(np.float64)
    return sx


def osnap_dense(x: np.ndarray, seed: int, r: int, s: int) -> np.ndarray:
    """OSNAP sketch S X (r x d, FP64) with s nonzeros +-1/sqrt(s) per column
    of S (block construction, streams.osnap_bucket_sign): for each hash j,
    SX[h_j(i)] += s_j(i) x_i over i ascending; the sums are then multiplied
    once by 1/sqrt(s). Block j's rows receive only hash j's rows, so every
    sketch row is an ascending-row sum, as in the CountSketch."""
    n, d = x.shape
    bucket, sign = streams.osnap_bucket_sign(seed, r, s, np.arange(n))
    sx = np.zeros((r, d), dtype=np.float64)
    xf = np.asarray(x, dtype=np.float64)
    for j in range(s):
        for i in range(n):
            sx[bucket[j, i]] += float(sign[j, i]) * xf[i]
    return sx * (1.0 / math.sqrt(s))


def osnap_csr(csr, seed: int, r: int, s: int) -> np.ndarray:
    """OSNAP sketch of a CSR matrix, same order as the dense form."""
    bucket, sign = streams.osnap_bucket_sign(seed, r, s, np.arange(csr.n))
    sx = np.zeros((r, csr.d), dtype=np.float64)
    rp = csr.row_ptr
    for j in range(s):
        for i in range(csr.n):
            a, b = int(rp[i]), int(rp[i + 1])
            if b > a:
                sx[bucket[j, i], csr.col_idx[a:b]] += float(sign[j, i]) * \
                    csr.val[a:b].astype(np.float64)
    return sx * (1.0 / math.sqrt(s))


def srht_plan(seed: int, n: int, r: int):
    """(n', rows): the padded length n' = 2^ceil(log2 n) and the r sampled
    Hadamard rows, in sketch-row order."""
    n2 = 1 << max(0, (n - 1).bit_length())
    if r > n2:
        raise ValueError("SRHT needs r <= n' (the padded row count)")
    w0, _ = streams.sample_words(seed, streams.STREAM_SRHT_ROWS, 0,
                                 np.arange(n2))
    return n2, np.argsort(w0.astype(np.uint64), kind="stable")[:r]


def srht_signs(seed: int, n: int) -> np.ndarray:
    h = streams.poly_hash(streams.hash_coeffs(seed, streams.STREAM_SRHT_SIGN),
                          np.arange(n))
    return np.array([1 - 2 * (int(v) & 1) for v in h], dtype=np.float64)


def fwht_rows(y: np.ndarray) -> np.ndarray:
    """Unnormalised Walsh-Hadamard transform along the rows (length a power
    of two), Sylvester order: stage b = 0, 1, ... replaces rows a and
    a + 2^b (bit b of a clear) by their sum and difference."""
    n2, d = y.shape
    y = y.copy()
    h = 1
    while h < n2:
        v = y.reshape(n2 // (2 * h), 2, h, d)
        a = v[:, 0].copy()
        b = v[:, 1].copy()
        v[:, 0] = a + b
        v[:, 1] = a - b
        h *= 2
    return y


def srht_dense(x: np.ndarray, seed: int, r: int) -> np.ndarray:
    """SRHT sketch S X = (1/sqrt(r)) P H D X (r x d, FP64): D the random
    signs, X padded with zero rows to n', H the unnormalised Hadamard
    transform, P the r sampled rows; the 1/sqrt(r) is applied once at the end
    (E[S^T S] = I)."""
    n, d = x.shape
    n2, rows = srht_plan(seed, n, r)
    y = np.zeros((n2, d), dtype=np.float64)
    y[:n] = srht_signs(seed, n)[:, None] * np.asarray(x, dtype=np.float64)
    return fwht_rows(y)[rows] * (1.0 / math.sqrt(r))


def gaussian_sketch_dense(x: np.ndarray, seed: int, r: int,
                          g: np.ndarray | None = None,
                          precision: str = "f64") -> np.ndarray:
    """SX = G X / sqrt(r) in FP64.

    ``precision`` selects the entries of G: "f64" the FP64 Box-Muller stream,
    "f32" the FP32 generator (plain FP32 path), "bf16" and "fp8" the quantile
    form rounded to BF16 or e4m3 (BF16 and FP8 inputs). The product is FP64.
    """
    n = x.shape[0]
    if g is None:
        if precision == "f64":
            g = streams.gaussian_sketch_matrix(seed, r, n)
        elif precision == "f32":
            g = streams.gaussian_sketch_matrix_f32(seed, r, n)
        elif precision in ("bf16", "fp8"):
            g = streams.gaussian_sketch_matrix_q(seed, r, n, precision)
        else:
            raise ValueError(precision)
    return (np.asarray(g, dtype=np.float64) @ np.asarray(x, dtype=np.float64)) \
        / math.sqrt(r)
