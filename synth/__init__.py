"""Seeded synthetic inputs shaped like the workloads of Chin & Liang (ACML 2018).

This module only draws input matrices. It holds none of the leverage-score
arithmetic: the sketch, the factorisations and the scores live elsewhere (the
HIP library and, separately, the CPU oracle), and both read their inputs from
here. Every generator is a pure function of its seed (numpy PCG64).

Shapes and distributions:

* ``lowrank_dense`` -- X = diag(rho) (U diag(sigma) V^T + E) with U, V Haar
  (QR of a Gaussian with the sign fix of Mezzadri 2007), E Gaussian noise and
  rho log-normal row scales, so leverage is non-uniform. ``config0`` uses
  n=20000, d=64, rank 32, sigma_j = 2^(-j/4), noise std 1e-3, rho = e^N(0,1).
* ``image_like`` -- stands in for a 60000 x 784 image matrix (the paper's
  MNIST experiment; the dataset itself is not used): entries clipped to [0, 1]
  from 0.5 + alpha * Z W^T + N(0, 0.02^2), Z drawn from 10 Gaussian clusters in
  a 50-dim latent space, W Haar 784 x 50, alpha chosen so the pre-clip spread
  is 0.25.
* ``text_like_csr`` -- stands in for a bag-of-words/tf-idf matrix: n rows over
  d columns, row nnz log-normal (mean about 0.5 % of d), column ranks drawn
  from Zipf(1.1) truncated to d and mapped through a seeded permutation,
  duplicate draws merged, values log(1 + c) * idf_j with c a zero-truncated
  Poisson(2) count.
* ``precision_dense`` -- rank-256 signal with sigma_j = j^-1.5 in d=512,
  noise 1e-4, row scales e^N(0, 1.5^2) (the reduced-precision workload).
* ``serving_pool`` / ``serving_jobs`` -- the serving workload: a Poisson
  stream of jobs with n log-uniform in [1e4, 2e6], d from {64, ..., 1024},
  FP32 or BF16, each a row window of one of ten base matrices (one per d and
  dtype, 2e6 rows, drawn on the device like the plain small workload) with
  its own sketch seed.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "haar", "lowrank_dense", "config0", "image_like", "config1",
    "text_like_csr", "config2", "precision_dense", "to_bf16_bits",
    "bf16_bits_to_f64", "to_fp8_e4m3", "fp8_e4m3_to_f64", "Csr",
    "lowrank_dense_device", "serving_pool", "serving_jobs",
    "precision_dense_device", "to_fp8_e4m3_device",
]


def haar(rng: np.random.Generator, n: int, k: int) -> np.ndarray:
    """n x k matrix with orthonormal columns, Haar-distributed (n >= k)."""
    g = rng.standard_normal((n, k))
    q, r = np.linalg.qr(g)
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s


def lowrank_dense(n: int, d: int, rank: int, sigma: np.ndarray, noise: float,
                  row_sigma: float, seed: int) -> np.ndarray:
    """FP64 X = diag(rho) (U diag(sigma) V^T + E)."""
    rng = np.random.default_rng(seed)
    u = haar(rng, n, rank)
    v = haar(rng, d, rank)
    x = (u * sigma[None, :]) @ v.T
    if noise > 0:
        x += noise * rng.standard_normal((n, d))
    if row_sigma > 0:
        rho = np.exp(row_sigma * rng.standard_normal(n))
        x *= rho[:, None]
    return x


def config0(n: int = 20000, d: int = 64, seed: int = 1000) -> np.ndarray:
    """Plain method, small: dense FP64, rank d/2, sigma_j = 2^(-j/4)."""
    rank = d // 2
    sigma = 2.0 ** (-np.arange(rank) / 4.0)
    return lowrank_dense(n, d, rank, sigma, 1e-3, 1.0, seed)


def image_like(n: int, d: int, latent: int = 50, clusters: int = 10,
               seed: int = 1001) -> np.ndarray:
    """FP32 image-like matrix in [0, 1] (see module docstring)."""
    rng = np.random.default_rng(seed)
    mu = rng.standard_normal((clusters, latent))
    c = rng.integers(0, clusters, n)
    z = mu[c] + 0.5 * rng.standard_normal((n, latent))
    w = haar(rng, d, latent)
    s = z @ w.T
    alpha = 0.25 / s.std()
    x = 0.5 + alpha * s + 0.02 * rng.standard_normal((n, d))
    return np.clip(x, 0.0, 1.0).astype(np.float32)


def config1(n: int = 60000, d: int = 784, seed: int = 1001) -> np.ndarray:
    return image_like(n, d, seed=seed)


class Csr:
    """Plain CSR triple (row_ptr int64[n+1], col_idx int32[nnz], val)."""

    def __init__(self, n, d, row_ptr, col_idx, val):
        self.n, self.d = int(n), int(d)
        self.row_ptr = row_ptr
        self.col_idx = col_idx
        self.val = val

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_dense(self, dtype=np.float64) -> np.ndarray:
        x = np.zeros((self.n, self.d), dtype=dtype)
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        x[rows, self.col_idx] = self.val
        return x


def text_like_csr(n: int, d: int, density: float = 0.005, zipf_s: float = 1.1,
                  seed: int = 1002) -> Csr:
    """Sparse tf-idf-like FP32 CSR matrix (see module docstring)."""
    rng = np.random.default_rng(seed)
    mean_nnz = density * d
    mu = math.log(mean_nnz) - 0.5
    m = np.rint(np.exp(mu + rng.standard_normal(n))).astype(np.int64)
    m = np.clip(m, 1, d)
    # Zipf(s) over ranks 1..d, inverse CDF sampling
    p = np.arange(1, d + 1, dtype=np.float64) ** (-zipf_s)
    cdf = np.cumsum(p)
    cdf /= cdf[-1]
    total = int(m.sum())
    ranks = np.searchsorted(cdf, rng.random(total), side="right")
    ranks = np.minimum(ranks, d - 1)
    perm = rng.permutation(d)
    cols = perm[ranks].astype(np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), m)
    key = np.unique(rows * d + cols)          # merge duplicate draws, sort
    rows = key // d
    cols = (key % d).astype(np.int32)
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    df = np.bincount(cols, minlength=d).astype(np.float64)
    idf = np.log(n / (1.0 + df))
    # zero-truncated Poisson(2) by rejection of zeros
    c = rng.poisson(2.0, key.size)
    while True:
        z = c == 0
        if not z.any():
            break
        c[z] = rng.poisson(2.0, int(z.sum()))
    val = (np.log1p(c) * idf[cols]).astype(np.float32)
    return Csr(n, d, row_ptr, cols, val)


def config2(n: int = 500000, d: int = 4096, seed: int = 1002) -> Csr:
    return text_like_csr(n, d, seed=seed)


def precision_dense(n: int = 4_000_000, d: int = 512, rank: int = 256,
                    seed: int = 1003) -> np.ndarray:
    """FP64 rank-256 signal, sigma_j = j^-1.5, noise 1e-4, rho = e^N(0,1.5^2)."""
    sigma = np.arange(1, rank + 1, dtype=np.float64) ** -1.5
    return lowrank_dense(n, d, rank, sigma, 1e-4, 1.5, seed)


def to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round FP32/FP64 values to bfloat16 (round to nearest even); uint16 bits."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) >> 16
    return u.astype(np.uint16)


def bf16_bits_to_f64(b: np.ndarray) -> np.ndarray:
    """Exact decode of bfloat16 bit patterns."""
    u = (np.asarray(b, dtype=np.uint32) << 16).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


# Non-negative finite values of the OCP fp8 e4m3fn format, by code 0 .. 126
# (code 127 is NaN): subnormals m 2^-9, normals (1 + m/8) 2^(e-7).
_E4M3 = np.array([(m * 2.0 ** -9) if e == 0 else (1.0 + m / 8.0) * 2.0 ** (e - 7)
                  for e in range(16) for m in range(8)][:127])


def to_fp8_e4m3(x: np.ndarray):
    """Quantise a dense matrix to fp8 e4m3fn with one FP32 scale per column.

    The scale of column j is max_i |x_ij| / 448 (1 for an all-zero column);
    codes round x_ij / scale_j to the nearest representable value, ties to the
    even code. Returns (codes uint8 n x d, col_scale float32 d); the value a
    code stands for is ``fp8_e4m3_to_f64(codes, col_scale)``.
    """
    xf = np.asarray(x, dtype=np.float64)
    cm = np.abs(xf).max(axis=0)
    cs = np.where(cm > 0, cm / 448.0, 1.0).astype(np.float32)
    v = xf / cs.astype(np.float64)[None, :]
    a = np.minimum(np.abs(v), 448.0)
    hi = np.searchsorted(_E4M3, a, side="left").clip(0, 126)
    lo = (hi - 1).clip(0, 126)
    dl, dh = a - _E4M3[lo], _E4M3[hi] - a
    pick_hi = (dh < dl) | ((dh == dl) & (hi % 2 == 0))
    code = np.where(pick_hi, hi, lo).astype(np.uint8)
    code |= np.where((v < 0) & (code != 0), 0x80, 0).astype(np.uint8)
    return code, cs


def fp8_e4m3_to_f64(codes: np.ndarray, col_scale: np.ndarray) -> np.ndarray:
    """Exact value of e4m3fn codes times their FP32 column scales (FP64)."""
    c = np.asarray(codes, dtype=np.uint8)
    mag = _E4M3[np.minimum(c & 0x7F, 126)]
    mag = np.where((c & 0x7F) == 127, np.nan, mag)
    val = np.where(c & 0x80, -mag, mag)
    return val * np.asarray(col_scale, dtype=np.float64)[None, :]


def lowrank_dense_device(n: int, d: int, rank: int, sigma, noise: float,
                         row_sigma: float, seed: int, device="cuda",
                         chunk: int = 1 << 18):
    """``lowrank_dense`` drawn on a torch device (FP64), for inputs too large
    to draw on the host in reasonable time: U Haar (QR of a Gaussian with the
    sign fix), V Haar, Gaussian noise and log-normal row scales, all from one
    seeded torch generator. Same distribution as ``lowrank_dense``, different
    random numbers."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)

    def haar_t(m, k):
        a = torch.randn(m, k, generator=g, device=device, dtype=torch.float64)
        q, r = torch.linalg.qr(a)
        s = torch.sign(torch.diagonal(r))
        s[s == 0] = 1.0
        return q * s

    u = haar_t(n, rank)
    v = haar_t(d, rank)
    sv = torch.as_tensor(np.asarray(sigma, dtype=np.float64), device=device)
    w = (v * sv[None, :]).T.contiguous()          # rank x d
    x = torch.empty(n, d, device=device, dtype=torch.float64)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        blk = u[a:b] @ w
        if noise > 0:
            blk += noise * torch.randn(b - a, d, generator=g, device=device,
                                       dtype=torch.float64)
        x[a:b] = blk
    del u
    if row_sigma > 0:
        rho = torch.exp(row_sigma * torch.randn(n, generator=g, device=device,
                                                dtype=torch.float64))
        x *= rho[:, None]
    return x


def serving_pool(d_values=(64, 128, 256, 512, 1024), n: int = 2_000_000,
                 seed: int = 1004, device="cuda"):
    """Base matrices of the serving workload, one per (d, dtype), FP32 and
    BF16 torch tensors on ``device``: rank d/2, sigma_j = 2^(-j/4), noise
    1e-3, row scales e^N(0,1) (the plain small recipe at larger n). A job is a
    seeded window of rows of one of them."""
    import torch
    pool = {}
    for i, d in enumerate(d_values):
        rank = d // 2
        sigma = 2.0 ** (-np.arange(rank) / 4.0)
        x = lowrank_dense_device(n, d, rank, sigma, 1e-3, 1.0, seed + 17 * i,
                                 device)
        pool[(d, "f32")] = x.to(torch.float32)
        pool[(d, "bf16")] = x.to(torch.bfloat16)
        del x
    return pool


def serving_jobs(n_jobs: int = 1024, rate: float = 200.0, seed: int = 1005,
                 n_lo: float = 1e4, n_hi: float = 2e6,
                 d_values=(64, 128, 256, 512, 1024), pool_n: int = 2_000_000):
    """Job descriptors of the serving workload: Poisson arrivals at ``rate``
    jobs/s, n log-uniform in [n_lo, n_hi], d uniform over ``d_values``,
    FP32/BF16 with equal odds, r = d * U{4..8}, k = 32, a row window of the
    pool matrix and a per-job sketch seed."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n_jobs))
    jobs = []
    for j in range(n_jobs):
        n = int(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))
        n = min(n, pool_n)
        d = int(rng.choice(d_values))
        dt = "f32" if rng.random() < 0.5 else "bf16"
        row0 = int(rng.integers(0, pool_n - n + 1))
        r = d * int(rng.integers(4, 9))
        jobs.append({"arrival_s": float(t[j]), "n": n, "d": d, "dtype": dt,
                     "row0": row0, "r": r, "k": 32,
                     "seed": 3_000_000 + j})
    return jobs


def precision_dense_device(n: int = 4_000_000, d: int = 512, rank: int = 256,
                           seed: int = 1003, device="cuda"):
    """``precision_dense`` drawn on a torch device (FP64 tensor): the same
    recipe (sigma_j = j^-1.5, noise 1e-4, rho = e^N(0, 1.5^2)) from a seeded
    torch generator, for the full-size precision workload (4e6 x 512 FP64 is
    16 GB, slow to draw and to move from the host)."""
    sigma = np.arange(1, rank + 1, dtype=np.float64) ** -1.5
    return lowrank_dense_device(n, d, rank, sigma, 1e-4, 1.5, seed, device)


def to_fp8_e4m3_device(x):
    """``to_fp8_e4m3`` of a torch tensor on its own device: per-column FP32
    scales max |x_j| / 448 (1 for a zero column) and e4m3fn codes of x / scale
    rounded to nearest even (torch's float8_e4m3fn conversion, which the
    host quantiser matches). Returns (codes uint8, col_scale float32)."""
    import torch
    cm = x.abs().amax(dim=0).to(torch.float64)
    cs = torch.where(cm > 0, cm / 448.0, torch.ones_like(cm)).to(torch.float32)
    codes = torch.empty(x.shape, dtype=torch.uint8, device=x.device)
    step = max(1, (1 << 26) // max(1, x.shape[1]))
    for a in range(0, x.shape[0], step):
        v = x[a:a + step].to(torch.float64) / cs.to(torch.float64)[None, :]
        codes[a:a + step] = v.to(torch.float8_e4m3fn).view(torch.uint8)
    return codes, cs
