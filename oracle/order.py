"""Orderings of Algorithm 4 step 4 (policies of Sec. 5.2): "dec", "dec, swr"
and "dec, swor".

dec: rows by strictly decreasing leverage score; equal scores keep ascending
row index (a stable sort), which is the reading used for ties. The sampling
policies draw from P_i = L_i / sum_j L_j (Algorithm 4 step 3), below.
"""
from __future__ import annotations

import math

import numpy as np


def dec_order(scores) -> np.ndarray:
    """Permutation p with scores[p[0]] the largest; ties by ascending index."""
    s = np.asarray(scores)
    idx = list(range(s.shape[0]))
    # plain stable sort on the key (-score); Python's sort is stable
    idx.sort(key=lambda i: -float(s[i]))
    return np.asarray(idx, dtype=np.int64)


# --------------------------------------------------------------------------
# Sampling policies of Algorithm 4 step 4 (Sec. 5.2): dec-swr and dec-swor
# --------------------------------------------------------------------------
# P_i = L_i / sum_j L_j (Algorithm 4 step 3). Readings (also in the design
# notes): a score that is not a positive finite number has probability 0;
# each epoch draws afresh from the seeded stream of that epoch.
#
# dec-swr: n draws with replacement from P, in draw order. P is represented
# exactly by integer weights w_i = floor(L_i 2^(30 - e)) with 2^(e-1) <= max L
# < 2^e, so the cumulative weights C_i = w_0 + ... + w_i are exact integers
# (W = C_{n-1} < n 2^30); draw t takes the 53-bit integer m_t of its stream and
# picks the smallest i with C_i > floor(m_t W / 2^53) (inverse transform).
#
# dec-swor: a weighted random permutation without replacement, in draw order
# (successive draws proportional to P among the rows not yet drawn), by the
# exponential keys of Efraimidis and Spirakis: key_i = E_i / L_i with
# E_i = 0 - ln u_i exponential, rows in ascending key, ties by ascending row; a
# row of probability 0 has key +inf. All of it in FP32, each operation
# rounded separately.
from . import streams  # noqa: E402


def _positive(s):
    s = np.asarray(s, dtype=np.float32)
    ok = np.isfinite(s) & (s > 0)
    return np.where(ok, s, np.float32(0.0)).astype(np.float32), ok


def swr_weights(scores) -> np.ndarray:
    """Integer weights w_i = floor(L_i 2^(30 - e)) (Python ints)."""
    s, ok = _positive(scores)
    if not ok.any():
        raise ValueError("no positive score")
    _, e = math.frexp(float(s.max()))
    return [int(math.floor(math.ldexp(float(v), 30 - e))) for v in s]


def swr_order(scores, seed: int, epoch: int) -> np.ndarray:
    """n row indices drawn with replacement with probability P_i."""
    w = swr_weights(scores)
    n = len(w)
    cum = np.cumsum(np.asarray(w, dtype=object)).astype(np.int64)
    total = int(cum[-1])
    w0, w1 = streams.sample_words(seed, streams.STREAM_SWR, epoch, np.arange(n))
    out = np.empty(n, dtype=np.int64)
    for t in range(n):
        m = ((int(w0[t]) << 32) | int(w1[t])) >> 11
        target = (m * total) >> 53
        out[t] = int(np.searchsorted(cum, target, side="right"))
    return out


def swor_keys(scores, seed: int, epoch: int) -> np.ndarray:
    """FP32 keys E_i / L_i (+inf for probability 0)."""
    s, ok = _positive(scores)
    n = s.shape[0]
    w0, _ = streams.sample_words(seed, streams.STREAM_SWOR, epoch, np.arange(n))
    # E = 0 - ln u (u = 1 gives +0, not -0)
    e = (np.float32(0.0) - streams.ln_f32(streams.unit_f32(w0))).astype(np.float32)
    with np.errstate(divide="ignore", invalid="ignore"):
        k = (e / np.where(ok, s, np.float32(1.0))).astype(np.float32)
    return np.where(ok, k, np.float32(np.inf)).astype(np.float32)


def swor_order(scores, seed: int, epoch: int) -> np.ndarray:
    """Permutation in ascending key order (ties by ascending row)."""
    k = swor_keys(scores, seed, epoch)
    idx = list(range(k.shape[0]))
    idx.sort(key=lambda i: float(k[i]))
    return np.asarray(idx, dtype=np.int64)
