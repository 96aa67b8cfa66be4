"""Seeded random streams, written from their published definitions.

The paper implements CountSketch "as a pair of hash functions" (Sec. 3.1.2)
without naming the family, and draws Gaussian sketches (Sec. 2.1) without
naming a generator. The readings used here (and, separately, by the GPU
library) are:

* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): state += 0x9E3779B97F4A7C15,
  then the 64-bit finaliser z ^= z>>30; z *= 0xBF58476D1CE4E5B9; z ^= z>>27;
  z *= 0x94D049BB133111EB; z ^= z>>31.
* Hash coefficients for stream ``s``: start from seed XOR (s * 0xD1B54A32D192ED03
  mod 2^64), draw four SplitMix64 outputs, reduce each mod p = 2^61 - 1.
* Degree-3 Carter-Wegman polynomial P(i) = a3 i^3 + a2 i^2 + a1 i + a0 mod p
  (4-wise independent over the prime field), evaluated by Horner's rule.
  Bucket h(i) = P_1(i) mod r; sign s(i) = +1 if P_2(i) is even, else -1.
* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): multipliers
  0xD2511F53, 0xCD9E8D57, Weyl key increments 0x9E3779B9, 0xBB67AE85.
* Gaussian entry (a, b) of stream s: one Philox block with counter
  (b >> 1, lo32(a), hi32(a), s) and key (lo32(seed), hi32(seed)); two 53-bit
  uniforms u1 = (m1 + 1) 2^-53 in (0, 1] from words (0, 1) and u2 = m2 2^-53
  from words (2, 3); Box-Muller z0 = sqrt(-2 ln u1) cos(2 pi u2),
  z1 = sqrt(-2 ln u1) sin(2 pi u2); entry (a, b) takes z0 if b is even.
  For the sketch S (r x n), a is the row index of X and b the sketch row; for
  Pi_2 (d x k), a is the row of Pi_2 and b its column.

* FP32 Gaussian sketch entry G[j][i] (``gaussian_f32``; stream 3): one
  Philox block per four consecutive data rows, counter (lo32(q), hi32(q), j, 3)
  with q = i >> 2, words (0, 1) for i mod 4 in {0, 1} and (2, 3) otherwise;
  u1 = ((w >> 8) + 1) 2^-24, u2 = (w' >> 8) 2^-24; Box-Muller with every step
  a separately rounded FP32 operation (ln by a degree-7 polynomial after a
  sqrt(2) range split, sqrt(L) = L rsqrt(L) with the 0x5F3759DF seed and three
  Newton steps, cos/sin of 2 pi u2 by quadrant: Taylor polynomials at the
  quadrant's centre rotated by +-sqrt(1/2)); cos for even i, sin for odd i.
  This is the plain FP32 path's generator.

* Quantile form of the Gaussian sketch entries (``gaussian_q``; stream 9),
  used for BF16 and FP8 inputs, whose sketch entries are BF16 or e4m3
  values: one Philox block per eight consecutive data rows, counter
  (lo32(q), hi32(q), j, 9) with q = i >> 3; data row i takes the 16-bit half
  (i & 1: high, else low) of word (i >> 1) & 3. Its top bit is the sign and
  its low 15 bits a cell m of 2^15 equiprobable cells of |Z|, Z standard
  normal; the magnitude is the cell's midpoint quantile
  t_m = sqrt(2) erfinv((2 m + 1) / 65536) rounded to BF16 (ties to even) for
  BF16 input, to e4m3 (ties to even) for FP8 input. Every t_m lies more than
  1e-9 of itself from a rounding boundary of either format, so any FP64
  evaluation of erfinv good to 1e-12 gives the same two tables.

Stream ids: 1 bucket hash, 2 sign hash, 3 Gaussian sketch (FP32 entries),
4 Pi_2, 5 dec-swr draws, 6 dec-swor keys, 7 SRHT signs, 8 SRHT row choice,
9 Gaussian sketch (quantile form).

* SRHT (the randomized Hadamard transform of Sec. 2.1 / Table 1): row i's
  sign is +1 if P(i) is even for the polynomial hash of stream 7; the r
  sampled rows of the n' = 2^ceil(log2 n) Hadamard rows are those with the r
  smallest 32-bit words w0 of the sampling block (counter (lo32(i), hi32(i),
  0, 8)), ties by ascending row, in that order.

* Sampling draws (the dec-swr / dec-swor policies of Algorithm 4 step 4):
  for item t and epoch, one Philox4x32-10 block with counter (lo32(t),
  hi32(t), epoch, stream) and key (lo32(seed), hi32(seed)). dec-swr takes the
  53-bit integer ((w0 << 32) | w1) >> 11; dec-swor the FP32 unit
  u = ((w0 >> 8) + 1) 2^-24 and E = 0 - ln u with the FP32 logarithm of the
  Gaussian generator.

* OSNAP with s nonzeros per column (the sparse embedding the paper lists
  beside CountSketch in Sec. 2.1 and implements, like CountSketch, as hash
  functions in Sec. 3.1.2), block construction: the r sketch rows form s
  blocks of b = r / s rows; hash j < s puts row i into block j at
  j b + (P_1j(i) mod b) with sign from the parity of P_2j(i). Hash 0 uses
  streams 1 and 2 (so s = 1 is CountSketch); hash j >= 1 uses streams
  16 + 2j (bucket) and 17 + 2j (sign).
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
MASK32 = 0xFFFFFFFF
P61 = (1 << 61) - 1

STREAM_BUCKET = 1
STREAM_SIGN = 2
STREAM_GAUSS_S = 3
STREAM_PI2 = 4
STREAM_SWR = 5
STREAM_SWOR = 6
STREAM_SRHT_SIGN = 7
STREAM_SRHT_ROWS = 8
STREAM_GAUSS_Q = 9


def splitmix64_mix(z: int) -> int:
    """SplitMix64 output finaliser on a 64-bit integer."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def splitmix64_sequence(state: int, count: int) -> list[int]:
    """First ``count`` SplitMix64 outputs from ``state``."""
    out = []
    for _ in range(count):
        state = (state + 0x9E3779B97F4A7C15) & MASK64
        out.append(splitmix64_mix(state))
    return out


def hash_coeffs(seed: int, stream: int) -> list[int]:
    """(a0, a1, a2, a3) of the degree-3 polynomial hash for ``stream``."""
    state = (seed ^ ((stream * 0xD1B54A32D192ED03) & MASK64)) & MASK64
    return [z % P61 for z in splitmix64_sequence(state, 4)]


def poly_hash(coeffs: list[int], idx) -> np.ndarray:
    """P(i) mod 2^61-1 for every i in ``idx`` (exact Python-integer arithmetic)."""
    a0, a1, a2, a3 = coeffs
    i = np.asarray(idx, dtype=np.int64).astype(object)
    acc = (a3 * i + a2) % P61
    acc = (acc * i + a1) % P61
    acc = (acc * i + a0) % P61
    return acc


def bucket_sign(seed: int, r: int, idx) -> tuple[np.ndarray, np.ndarray]:
    """CountSketch bucket h(i) in [0, r) and sign s(i) in {+1, -1}."""
    hb = poly_hash(hash_coeffs(seed, STREAM_BUCKET), idx)
    hs = poly_hash(hash_coeffs(seed, STREAM_SIGN), idx)
    bucket = np.array([int(v) % r for v in hb], dtype=np.int64)
    sign = np.array([1 - 2 * (int(v) & 1) for v in hs], dtype=np.int64)
    return bucket, sign


def osnap_streams(j: int) -> tuple[int, int]:
    """(bucket stream, sign stream) of OSNAP hash j."""
    if j == 0:
        return STREAM_BUCKET, STREAM_SIGN
    return 16 + 2 * j, 17 + 2 * j


def osnap_bucket_sign(seed: int, r: int, s: int, idx):
    """OSNAP buckets and signs, each s x len(idx): hash j sends row i to
    j (r // s) + (P_1j(i) mod (r // s)) with sign +1 if P_2j(i) is even."""
    if s < 1 or r % s != 0:
        raise ValueError("OSNAP needs s >= 1 dividing r")
    b = r // s
    idx = np.asarray(idx, dtype=np.int64)
    buckets = np.empty((s, idx.shape[0]), dtype=np.int64)
    signs = np.empty((s, idx.shape[0]), dtype=np.int64)
    for j in range(s):
        sb, ss = osnap_streams(j)
        hb = poly_hash(hash_coeffs(seed, sb), idx)
        hs = poly_hash(hash_coeffs(seed, ss), idx)
        buckets[j] = [j * b + int(v) % b for v in hb]
        signs[j] = [1 - 2 * (int(v) & 1) for v in hs]
    return buckets, signs


# --------------------------------------------------------------------------
# Philox4x32-10
# --------------------------------------------------------------------------
_PHILOX_M0 = 0xD2511F53
_PHILOX_M1 = 0xCD9E8D57
_PHILOX_W0 = 0x9E3779B9
_PHILOX_W1 = 0xBB67AE85


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32 with 10 rounds on arrays of 32-bit counter words.

    Returns the four 32-bit output words as uint64 arrays.
    """
    c0 = np.asarray(c0, dtype=np.uint64) & MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & MASK32
    k0 = np.uint64(k0 & MASK32)
    k1 = np.uint64(k1 & MASK32)
    m0 = np.uint64(_PHILOX_M0)
    m1 = np.uint64(_PHILOX_M1)
    lo_mask = np.uint64(MASK32)
    sh = np.uint64(32)
    for rnd in range(10):
        if rnd > 0:
            k0 = np.uint64((int(k0) + _PHILOX_W0) & MASK32)
            k1 = np.uint64((int(k1) + _PHILOX_W1) & MASK32)
        p0 = c0 * m0            # < 2^64, exact in uint64
        p1 = c2 * m1
        hi0, lo0 = p0 >> sh, p0 & lo_mask
        hi1, lo1 = p1 >> sh, p1 & lo_mask
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def gaussian(seed: int, stream: int, a, b) -> np.ndarray:
    """Standard normal entry (a, b) of ``stream`` (arrays broadcast), FP64."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a, b = np.broadcast_arrays(a, b)
    w0, w1, w2, w3 = philox4x32_10(b >> np.uint64(1), a & np.uint64(MASK32),
                                   a >> np.uint64(32),
                                   np.full(a.shape, stream, dtype=np.uint64),
                                   seed & MASK32, (seed >> 32) & MASK32)
    m1 = (w0 << np.uint64(21)) | (w1 >> np.uint64(11))
    m2 = (w2 << np.uint64(21)) | (w3 >> np.uint64(11))
    m1 &= np.uint64((1 << 53) - 1)
    m2 &= np.uint64((1 << 53) - 1)
    u1 = (m1.astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = m2.astype(np.float64) * 2.0 ** -53
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    odd = (b & np.uint64(1)).astype(bool)
    return np.where(odd, rad * np.sin(ang), rad * np.cos(ang))


def pi2_matrix(seed: int, d: int, k: int) -> np.ndarray:
    """Second JL projection Pi_2 (d x k), entries N(0, 1/k)."""
    j = np.arange(d, dtype=np.uint64)[:, None]
    c = np.arange(k, dtype=np.uint64)[None, :]
    return gaussian(seed, STREAM_PI2, j, c) / np.sqrt(k)


def gaussian_sketch_matrix(seed: int, r: int, n: int) -> np.ndarray:
    """Gaussian sketch G (r x n), entries N(0, 1) (the 1/sqrt(r) is applied
    to the sketch product, not here)."""
    i = np.arange(n, dtype=np.uint64)[None, :]
    j = np.arange(r, dtype=np.uint64)[:, None]
    return gaussian(seed, STREAM_GAUSS_S, i, j)


def sample_words(seed: int, stream: int, epoch: int, t):
    """Philox words (w0, w1) of sampling item t (uint64 arrays)."""
    t = np.asarray(t, dtype=np.uint64)
    w0, w1, _, _ = philox4x32_10(t & np.uint64(MASK32), t >> np.uint64(32),
                                 np.full(t.shape, epoch, np.uint64),
                                 np.full(t.shape, stream, np.uint64),
                                 seed & MASK32, (seed >> 32) & MASK32)
    return w0, w1


# --------------------------------------------------------------------------
# FP32 Gaussian entries of the sketch matrix S (the reduced-precision path)
# --------------------------------------------------------------------------
# Definition (shared with the GPU by specification only): for data row i and
# sketch row j, one Philox4x32-10 block with counter (lo32(i >> 2),
# hi32(i >> 2), j, stream) and key (lo32(seed), hi32(seed)) gives four 32-bit
# words; words (0, 1) make a Box-Muller pair for rows i = 4q, 4q+1 and words
# (2, 3) one for 4q+2, 4q+3. Every step below is a separately rounded FP32
# operation (no fused multiply-add), so the value is reproducible bit for bit:
#   u1 = ((w >> 8) + 1) 2^-24 in (0, 1],  u2 = (w' >> 8) 2^-24 in [0, 1)
#   ln u1 = e ln2 + t q(t), u1 = 2^e m, m in [sqrt(1/2), sqrt(2)), t = m - 1,
#           q a degree-7 least-squares fit of ln(1+t)/t (coefficients below)
#   rad = L y with L = -2 ln u1 and y = 1/sqrt(L) from the bit-level initial
#         guess 0x5F3759DF - (bits(L) >> 1) refined by three Newton steps
#         (rad = 0 when L = 0)
#   angle 2 pi u2 = (2k+1) pi/4 + x, k = floor(4 u2), x = (4 u2 - k - 1/2) pi/2,
#         cos x, sin x by Taylor polynomials to x^8 / x^9, rotated by the
#         quadrant angle with sqrt(1/2) factors
#   z = rad cos(angle), z' = rad sin(angle).
F32 = np.float32
_LN_Q = [F32(0.9999999403953552), F32(-0.5000036358833313),
         F32(0.33335113525390625), F32(-0.24970071017742157),
         F32(0.19898565113544464), F32(-0.17247013747692108),
         F32(0.1623418927192688), F32(-0.10134056955575943)]
_LN2 = F32(0.6931471824645996)
_SQRT2 = F32(1.4142135381698608)
_HALF_PI = F32(1.5707963705062866)
_RSQRT_HALF = F32(0.7071067690849304)
_COS_T = [F32(1.0 / 40320.0), F32(-1.0 / 720.0), F32(1.0 / 24.0), F32(-0.5)]
_SIN_T = [F32(1.0 / 362880.0), F32(-1.0 / 5040.0), F32(1.0 / 120.0),
          F32(-1.0 / 6.0)]


def unit_f32(w):
    """u = ((w >> 8) + 1) 2^-24 in (0, 1] from 32-bit words (uint64 arrays)."""
    ua = (np.asarray(w, dtype=np.uint64) >> np.uint64(8)).astype(np.uint32)
    return (ua.astype(F32) + F32(1.0)) * F32(2.0 ** -24)


def ln_f32(u1):
    """ln u for FP32 u in (0, 1], separately rounded FP32 operations: u =
    2^e m with m in [sqrt(1/2), sqrt(2)), ln u = e ln2 + t q(t), t = m - 1."""
    u1 = np.asarray(u1, dtype=F32)
    bits = u1.view(np.uint32)
    e = (bits >> np.uint32(23)).astype(np.int32) - 127
    m = ((bits & np.uint32(0x7FFFFF)) | np.uint32(0x3F800000)).view(F32)
    big = m > _SQRT2
    m = np.where(big, m * F32(0.5), m).astype(F32)
    e = np.where(big, e + 1, e)
    t = m - F32(1.0)
    q = _LN_Q[7]
    for c in _LN_Q[6::-1]:
        q = q * t
        q = q + c
    lnm = t * q
    ln_u = e.astype(F32) * _LN2
    return (ln_u + lnm).astype(F32)


def _box_muller_f32(wa, wb):
    """FP32 Box-Muller pair from two 32-bit words (arrays of uint64)."""
    ub = (wb >> np.uint64(8)).astype(np.uint32)
    two_m24 = F32(2.0 ** -24)
    u1 = unit_f32(wa)
    u2 = ub.astype(F32) * two_m24
    ln_u = ln_f32(u1)
    L = F32(-2.0) * ln_u
    # sqrt(L) = L / sqrt(L) via Newton steps on 1/sqrt(L)
    li = L.view(np.uint32)
    y = (np.uint32(0x5F3759DF) - (li >> np.uint32(1))).view(F32)
    hl = F32(0.5) * L
    for _ in range(3):
        y2 = y * y
        t2 = hl * y2
        t3 = F32(1.5) - t2
        y = y * t3
    rad = np.where(L == F32(0.0), F32(0.0), L * y).astype(F32)
    # angle
    q4 = u2 * F32(4.0)
    k = q4.astype(np.int32)
    f = q4 - k.astype(F32)
    x = (f - F32(0.5)) * _HALF_PI
    x2 = x * x
    c = _COS_T[0]
    for ct in _COS_T[1:]:
        c = c * x2
        c = c + ct
    cosx = c * x2
    cosx = cosx + F32(1.0)
    s = _SIN_T[0]
    for st in _SIN_T[1:]:
        s = s * x2
        s = s + st
    sinx = s * x2
    sinx = sinx * x
    sinx = sinx + x
    ca = np.where((k == 0) | (k == 3), _RSQRT_HALF, -_RSQRT_HALF).astype(F32)
    sa = np.where(k < 2, _RSQRT_HALF, -_RSQRT_HALF).astype(F32)
    cos_t = ca * cosx - sa * sinx
    sin_t = sa * cosx + ca * sinx
    return (rad * cos_t).astype(F32), (rad * sin_t).astype(F32)


def gaussian_f32(seed: int, stream: int, i, j) -> np.ndarray:
    """FP32 Gaussian entry for data row i and sketch row j (broadcast)."""
    i = np.asarray(i, dtype=np.uint64)
    j = np.asarray(j, dtype=np.uint64)
    i, j = np.broadcast_arrays(i, j)
    g = i >> np.uint64(2)
    w0, w1, w2, w3 = philox4x32_10(g & np.uint64(MASK32), g >> np.uint64(32),
                                   j, np.full(i.shape, stream, np.uint64),
                                   seed & MASK32, (seed >> 32) & MASK32)
    z0, z1 = _box_muller_f32(w0, w1)
    z2, z3 = _box_muller_f32(w2, w3)
    r = (i & np.uint64(3)).astype(np.int64)
    return np.select([r == 0, r == 1, r == 2], [z0, z1, z2], z3).astype(F32)


def gaussian_sketch_matrix_f32(seed: int, r: int, n: int, row0: int = 0):
    """Sketch G (r x n) with FP32 entries (the plain FP32 path), generated a
    few sketch rows at a time to bound the temporaries."""
    out = np.empty((r, n), dtype=F32)
    i = np.arange(row0, row0 + n, dtype=np.uint64)[None, :]
    step = max(1, (1 << 20) // max(n, 1))
    for j0 in range(0, r, step):
        j = np.arange(j0, min(r, j0 + step), dtype=np.uint64)[:, None]
        out[j0:j0 + j.shape[0]] = gaussian_f32(seed, STREAM_GAUSS_S, i, j)
    return out




# --------------------------------------------------------------------------
# Quantile form of the Gaussian sketch entries (BF16 and FP8 inputs)
# --------------------------------------------------------------------------
QCELLS = 1 << 15


def half_normal_quantiles() -> np.ndarray:
    """t_m = sqrt(2) erfinv((2 m + 1) / 65536), m = 0 .. 2^15 - 1 (FP64): the
    quantile of |Z| at the midpoint of the m-th of 2^15 equiprobable cells,
    since P(|Z| <= t) = erf(t / sqrt(2))."""
    from scipy.special import erfinv
    m = np.arange(QCELLS, dtype=np.float64)
    return np.sqrt(2.0) * erfinv((2.0 * m + 1.0) / 65536.0)


def round_to_format(v, fmt: str) -> np.ndarray:
    """Round non-negative FP64 values to the nearest BF16 ("bf16": 8
    significant bits) or OCP e4m3fn ("fp8": 4 significant bits, subnormal
    spacing 2^-9, largest finite 448) value, ties to even, as FP64."""
    v = np.asarray(v, dtype=np.float64)
    _, ex = np.frexp(v)                      # v = f 2^ex, f in [0.5, 1)
    e = ex - 1                               # v in [2^e, 2^(e+1))
    if fmt == "bf16":
        spacing = np.ldexp(1.0, e - 7)
    elif fmt == "fp8":
        spacing = np.ldexp(1.0, np.maximum(e, -6) - 3)
    else:
        raise ValueError(fmt)
    out = np.round(v / spacing) * spacing    # exact quotient; half to even
    out = np.where(v == 0.0, 0.0, out)
    if fmt == "fp8":
        out = np.minimum(out, 448.0)
    return out


def quantile_table(fmt: str) -> np.ndarray:
    """Magnitudes of the quantile-form entries: t_m rounded to ``fmt``."""
    return round_to_format(half_normal_quantiles(), fmt)


def gaussian_q_halfwords(seed: int, i, j) -> np.ndarray:
    """The 16-bit value behind the quantile-form entry (data row i, sketch
    row j), broadcast, as int64."""
    i = np.asarray(i, dtype=np.uint64)
    j = np.asarray(j, dtype=np.uint64)
    i, j = np.broadcast_arrays(i, j)
    q = i >> np.uint64(3)
    w = philox4x32_10(q & np.uint64(MASK32), q >> np.uint64(32), j,
                      np.full(i.shape, STREAM_GAUSS_Q, np.uint64),
                      seed & MASK32, (seed >> 32) & MASK32)
    widx = ((i >> np.uint64(1)) & np.uint64(3)).astype(np.int64)
    word = np.select([widx == 0, widx == 1, widx == 2], list(w[:3]), w[3])
    half = (i & np.uint64(1)).astype(bool)
    return np.where(half, word >> np.uint64(16),
                    word & np.uint64(0xFFFF)).astype(np.int64)


def gaussian_q(seed: int, i, j, fmt: str, table=None) -> np.ndarray:
    """Quantile-form Gaussian entry for data row i and sketch row j (FP64
    value of a BF16 or e4m3 number)."""
    t = quantile_table(fmt) if table is None else table
    v = gaussian_q_halfwords(seed, i, j)
    mag = t[v & (QCELLS - 1)]
    return np.where(v >> 15, -mag, mag)


def gaussian_sketch_matrix_q(seed: int, r: int, n: int, fmt: str,
                             row0: int = 0) -> np.ndarray:
    """Sketch G (r x n) with quantile-form entries (FP64 values). Each
    Philox block is evaluated once and split into its eight 16-bit halves
    (data rows 8q .. 8q + 7 in order), a few sketch rows at a time."""
    t = quantile_table(fmt)
    out = np.empty((r, n), dtype=np.float64)
    if n == 0:
        return out
    q0, q1 = row0 >> 3, (row0 + n - 1) >> 3
    q = np.arange(q0, q1 + 1, dtype=np.uint64)[None, :]
    lo = row0 - 8 * q0
    step = max(1, (1 << 18) // q.shape[1])
    for j0 in range(0, r, step):
        j = np.arange(j0, min(r, j0 + step), dtype=np.uint64)[:, None]
        jq, qq = np.broadcast_arrays(j, q)
        w = philox4x32_10(qq & np.uint64(MASK32), qq >> np.uint64(32), jq,
                          np.full(qq.shape, STREAM_GAUSS_Q, np.uint64),
                          seed & MASK32, (seed >> 32) & MASK32)
        halves = []
        for word in w:
            halves.append(word & np.uint64(0xFFFF))
            halves.append(word >> np.uint64(16))
        v = np.stack(halves, axis=-1).reshape(jq.shape[0], -1).astype(np.int64)
        v = v[:, lo:lo + n]
        mag = t[v & (QCELLS - 1)]
        out[j0:j0 + jq.shape[0]] = np.where(v >> 15, -mag, mag)
    return out
