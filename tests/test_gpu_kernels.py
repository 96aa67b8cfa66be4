"""GPU parity of every stage of the sketched leverage path against the CPU
oracle, through the C ABI (gfx950). Integer outputs (hash, bucket partition,
permutation) must be bit-exact; FP64 sketches of the same rows in the same
order are bit-exact as well; floating-point stages carry the tolerances
stated per test."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import leverage as olv
from oracle import metrics as omet
from oracle import order as oorder
from oracle import sketch as osk
from oracle import streams as ost

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def slso():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1812_07903_amd as m
    m.load_library()
    return m


@pytest.fixture(scope="module")
def ctx(slso):
    c = slso.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def csr_dev(slso, c):
    return slso.CsrMatrix(c.n, c.d, dev(c.row_ptr.astype(np.int64)),
                          dev(c.col_idx.astype(np.int32)),
                          dev(c.val.astype(np.float32)))


# ---- streams -----------------------------------------------------------------
@pytest.mark.parametrize("seed,r,row0,n", [
    (0, 1, 0, 1), (2025, 7, 0, 5003), (2025, 4096, 0, 20011),
    (2**63 + 5, 16384, 2**33 + 17, 4097), (77, 32768, 123456, 20000),
    (1002, 1000, 0, 3001)])
def test_hash_bit_exact(slso, seed, r, row0, n):
    b, s = slso.hash(seed, r, n, row0=row0)
    rb, rs = ost.bucket_sign(seed, r, np.arange(n) + row0)
    assert np.array_equal(host(b).astype(np.int64), rb)
    assert np.array_equal(host(s).astype(np.int64), rs)


@pytest.mark.parametrize("stream_id", [3, 4])
def test_gaussian_stream_matches(slso, stream_id):
    seed, rows, cols = 2**40 + 3, 301, 67
    z = host(slso.gaussian(seed, stream_id, rows, cols))
    ref = ost.gaussian(seed, stream_id, np.arange(rows)[:, None],
                       np.arange(cols)[None, :])
    assert np.max(np.abs(z - ref) / np.maximum(1.0, np.abs(ref))) < 1e-13


# ---- ordering ----------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 4095, 4096, 4097, 100003, 300001, 1100003])
def test_order_is_stable_descending(slso, ctx, n):
    rng = np.random.default_rng(n)
    s = rng.integers(0, 50, n).astype(np.float32) * np.float32(0.125)
    s[rng.integers(0, n, max(1, n // 10))] = 0.0
    perm = host(ctx.order(dev(s)))
    assert np.array_equal(perm.astype(np.int64), np.argsort(-s, kind="stable"))
    if n <= 5000:
        assert np.array_equal(perm.astype(np.int64), oorder.dec_order(s))


def test_order_all_equal_and_continuous(slso, ctx):
    assert np.array_equal(host(ctx.order(dev(np.full(9999, 3.5, np.float32)))),
                          np.arange(9999))
    s = np.random.default_rng(3).random(65537).astype(np.float32)
    perm = host(ctx.order(dev(s))).astype(np.int64)
    assert np.array_equal(perm, np.argsort(-s, kind="stable"))


# ---- sketches ----------------------------------------------------------------
def test_countsketch_dense_f64_bit_exact(slso, ctx):
    x = synth.config0(n=5000, d=64, seed=3)
    sx = host(ctx.sketch(dev(x), 11, 512))
    assert np.array_equal(sx, osk.countsketch_dense(x, 11, 512))


@pytest.mark.parametrize("n,d,r", [(3000, 100, 1024), (1, 1, 1), (777, 300, 1000),
                                   (5000, 784, 2048), (40, 3, 5),
                                   (20011, 256, 300), (9000, 512, 700),
                                   (4000, 1032, 1100), (50000, 64, 64)])
def test_countsketch_dense_f32_bit_exact(slso, ctx, n, d, r):
    """Bit-exact FP64 sums in ascending row order, for each width form of
    the fused kernel (one, two or four 4-element vectors per lane, 16, 8 or
    4 rows in flight) and for buckets of many rows (n / r near 800)."""
    if d >= 50:
        x = synth.image_like(n, d, seed=n + d)
    else:
        x = np.random.default_rng(n).random((n, d)).astype(np.float32)
    sx = host(ctx.sketch(dev(x), 5, r))
    assert np.array_equal(sx, osk.countsketch_dense(x, 5, r))


@pytest.mark.parametrize("n,d,r", [(4000, 48, 256), (7001, 600, 700)])
def test_countsketch_bf16_bit_exact(slso, ctx, n, d, r):
    x = synth.config0(n=n, d=d, seed=9)
    bits = synth.to_bf16_bits(x)
    xt = dev(bits.view(np.int16)).view(torch.bfloat16)
    sx = host(ctx.sketch(xt, 21, r))
    ref = osk.countsketch_dense(synth.bf16_bits_to_f64(bits), 21, r)
    assert np.array_equal(sx, ref)


@pytest.mark.parametrize("n,d,r", [(20000, 1500, 2048), (3000, 2500, 2500)])
def test_countsketch_csr_bit_exact(slso, ctx, n, d, r):
    c = synth.text_like_csr(n, d, density=0.01, seed=d)
    sx = host(ctx.sketch(csr_dev(slso, c), 8, r))
    assert np.array_equal(sx, osk.countsketch_csr(c, 8, r))


def _csr_rows(n, d, lengths, seed):
    """CSR with the given row lengths (distinct sorted columns per row)."""
    rng = np.random.default_rng(seed)
    cols = [np.sort(rng.choice(d, int(m), replace=False)) for m in lengths]
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum([len(c) for c in cols], out=row_ptr[1:])
    col_idx = np.concatenate(cols).astype(np.int32) if row_ptr[-1] else \
        np.zeros(0, np.int32)
    val = rng.standard_normal(col_idx.size).astype(np.float32)
    return synth.Csr(n, d, row_ptr, col_idx, val)


@pytest.mark.parametrize("n,d", [(9000, 4500), (8192, 4096), (30000, 300)])
def test_countsketch_csr_long_and_empty_rows(slso, ctx, n, d):
    """Rows of 0, 1, 63-65 and up to 300 entries (r = d); columns in one
    chunk (d <= 4096) or two (d = 4500, ragged second chunk); at d = 300
    about 100 rows per bucket (more than one group of 64): the sketch equals
    the oracle's bit for bit."""
    rng = np.random.default_rng(d)
    lengths = rng.choice([0, 1, 5, 63, 64, 65, 129, 300], size=n,
                         p=[0.15, 0.2, 0.25, 0.1, 0.1, 0.1, 0.05, 0.05])
    c = _csr_rows(n, d, np.minimum(lengths, d), seed=d + 1)
    sx = host(ctx.sketch(csr_dev(slso, c), 8, d))
    assert np.array_equal(sx, osk.countsketch_csr(c, 8, d))


def test_countsketch_csr_all_rows_empty(slso, ctx):
    """row_ptr all zero (one unused entry so that col_idx is not null): the
    sketch is zero and no entry is read."""
    n, d = 1000, 50
    x = slso.CsrMatrix(n, d, dev(np.zeros(n + 1, np.int64)),
                       dev(np.zeros(1, np.int32)), dev(np.ones(1, np.float32)))
    sx = host(ctx.sketch(x, 8, 64))
    assert sx.shape == (64, d) and not sx.any()


# ---- OSNAP ---------------------------------------------------------------------
@pytest.mark.parametrize("n,d,r,nnz", [(5000, 64, 512, 2), (3001, 33, 510, 3),
                                       (2000, 70, 1024, 4), (1, 1, 16, 16),
                                       (4000, 48, 256, 1)])
def test_osnap_dense_f64_bit_exact(slso, ctx, n, d, r, nnz):
    """S X with nnz signed nonzeros per column of S: FP64 sums in ascending
    row order per sketch row, times 1/sqrt(nnz) once."""
    x = synth.config0(n=n, d=d, seed=n + nnz) if n > 1 else np.ones((1, 1))
    sx = host(ctx.sketch(dev(x), 17, r, sketch=slso.OSNAP, nnz=nnz))
    assert np.array_equal(sx, osk.osnap_dense(x, 17, r, nnz))


def test_osnap_one_nonzero_is_countsketch(slso, ctx):
    x = synth.image_like(3000, 100, seed=3)
    a = host(ctx.sketch(dev(x), 9, 1024, sketch=slso.OSNAP, nnz=1))
    assert np.array_equal(a, host(ctx.sketch(dev(x), 9, 1024)))


def test_osnap_f32_and_csr_bit_exact(slso, ctx):
    x = synth.image_like(5000, 784, seed=5)
    sx = host(ctx.sketch(dev(x), 6, 2048, sketch=slso.OSNAP, nnz=2))
    assert np.array_equal(sx, osk.osnap_dense(x, 6, 2048, 2))
    c = synth.text_like_csr(20000, 1500, density=0.01, seed=8)
    sxc = host(ctx.sketch(csr_dev(slso, c), 8, 2048, sketch=slso.OSNAP, nnz=4))
    assert np.array_equal(sxc, osk.osnap_csr(c, 8, 2048, 4))


def test_osnap_rejects_bad_nnz(slso, ctx):
    x = dev(synth.config0(n=500, d=8, seed=1))
    for nnz, r in ((3, 64), (17, 68), (-2, 64)):
        with pytest.raises(slso.SlsoError) as ei:
            ctx.sketch(x, 1, r, sketch=slso.OSNAP, nnz=nnz)
        assert ei.value.status == slso.EINVAL


# ---- SRHT ----------------------------------------------------------------------
@pytest.mark.parametrize("n,d,r,f32", [(5000, 64, 512, False), (3000, 100, 1024, True),
                                       (1, 1, 1, False), (257, 5, 512, False),
                                       (70000, 64, 4096, True),
                                       (200, 7, 128, False), (40000, 96, 2048, True)])
def test_srht_bit_exact(slso, ctx, n, d, r, f32):
    """(1/sqrt(r)) P H D X: the same Sylvester stages in the same order as
    the oracle, so every FP64 value agrees exactly (passes of up to 8 stages:
    one, two and three passes, full and partial, here)."""
    x = synth.image_like(n, d, seed=n) if f32 else \
        (synth.config0(n=n, d=d, seed=n) if n > 1 else np.full((1, 1), 3.0))
    sx = host(ctx.sketch(dev(x), 29, r, sketch=slso.SRHT))
    assert np.array_equal(sx, osk.srht_dense(x, 29, r))


def test_srht_rejects_bad_arguments(slso, ctx):
    x = dev(synth.config0(n=500, d=8, seed=1))             # n' = 512
    with pytest.raises(slso.SlsoError) as ei:
        ctx.sketch(x, 1, 513, sketch=slso.SRHT)
    assert ei.value.status == slso.EINVAL
    c = synth.text_like_csr(1000, 50, seed=3)
    with pytest.raises(slso.SlsoError) as ei:
        ctx.sketch(csr_dev(slso, c), 1, 256, sketch=slso.SRHT)
    assert ei.value.status == slso.EUNSUPPORTED


# ---- QR ------------------------------------------------------------------------
@pytest.mark.parametrize("m,d", [(64, 64), (100, 37), (256, 32), (257, 33),
                                 (1000, 96), (3000, 200), (5000, 64),
                                 (70000, 40), (2048, 512), (16384, 784),
                                 (4099, 833), (1000, 140), (700, 257),
                                 (5000, 400), (12000, 2048), (4500, 4096)])
def test_qr_r_matches_householder(slso, ctx, m, d):
    """Cholesky-QR2 over the whole matrix (ragged row chunks and stripes,
    d below, at and past a multiple of 64; a last 128-column block of 1 to 16
    columns, whose Gram products the diagonal blocks form, or of more; Gram
    passes in the stream-K form: few blocks over few rows, 136 blocks at
    d = 2048, 528 at d = 4096 with ragged units)."""
    rng = np.random.default_rng(m * 7 + d)
    a = rng.standard_normal((m, d)) * np.exp(rng.standard_normal(d))[None, :]
    r, used = ctx.qr_r_path(dev(a.copy()))
    r = host(r)
    ref = olv.qr_r(a)
    assert used == slso.QR_CHOLQR2
    assert np.all(np.diag(r) >= 0) and np.all(np.tril(r, -1) == 0)
    err = np.abs(r - ref).max() / np.abs(ref).max()
    print(f"[qr cholqr2 {m}x{d}] rel err {err:.2e}", flush=True)
    assert err < 1e-12, err


@pytest.mark.parametrize("m,d", [(64, 64), (128, 64), (1000, 130), (3000, 200),
                                 (16384, 784), (70001, 128), (256, 256),
                                 (4096, 192)])
def test_qr_r_panel_path_matches_householder(slso, ctx, m, d):
    """The Householder path with 64-column Cholesky-QR2 panels (ragged row
    blocks, ragged trailing columns, d a multiple of 64, square)."""
    rng = np.random.default_rng(m + 3 * d)
    a = rng.standard_normal((m, d)) * np.exp(rng.standard_normal(d))[None, :]
    r, used = ctx.qr_r_path(dev(a.copy()), slso.QR_PANEL)
    r = host(r)
    ref = olv.qr_r(a)
    assert used == slso.QR_PANEL
    assert np.all(np.diag(r) >= 0) and np.all(np.tril(r, -1) == 0)
    err = np.abs(r - ref).max() / np.abs(ref).max()
    print(f"[qr panel {m}x{d}] rel err {err:.2e}", flush=True)
    assert err < 1e-12, err


@pytest.mark.parametrize("m,d", [(300, 37), (5000, 200)])
def test_qr_r_tree_path_matches_householder(slso, ctx, m, d):
    rng = np.random.default_rng(m + d)
    a = rng.standard_normal((m, d)) * np.exp(rng.standard_normal(d))[None, :]
    r, used = ctx.qr_r_path(dev(a.copy()), slso.QR_TREE)
    r = host(r)
    assert used == slso.QR_TREE
    ref = olv.qr_r(a)
    assert np.abs(r - ref).max() / np.abs(ref).max() < 1e-12


def _with_condition(kappa, m=3000, d=160, cols=None, seed=None):
    """m x d with condition number kappa: all columns (cols None), or only
    the first ``cols`` columns with the rest standard normal."""
    rng = np.random.default_rng(int(kappa) if seed is None else seed)
    c = d if cols is None else cols
    u, _ = np.linalg.qr(rng.standard_normal((m, c)))
    v, _ = np.linalg.qr(rng.standard_normal((c, c)))
    s = np.logspace(0, -np.log10(kappa), c)
    a = np.empty((m, d))
    a[:, :c] = (u * s) @ v.T
    a[:, c:] = rng.standard_normal((m, d - c))
    return a


@pytest.mark.parametrize("kappa,cols,path,expect", [
    (1e2, None, "auto", "cholqr2"), (1e5, None, "auto", "cholqr2_full"),
    (1e8, None, "auto", "panel_or_tree"), (1e2, 64, "panel", "panel"),
    (5e4, 64, "panel", "panel")])
def test_qr_r_ill_conditioned(slso, ctx, kappa, cols, path, expect):
    """Condition numbers that take each branch of the cascade: at 1e5 the
    first Cholesky-QR pass leaves G2 too far from I for the one-launch R2 and
    the blocked Cholesky runs; at 1e8 the whole-matrix Cholesky-QR2 does not
    apply and a Householder path takes over. On the panel path, a first
    panel with condition number 5e4 needs the blocked Cholesky in its second
    pass. R is compared through R^T R = A^T A (backward error), the
    meaningful measure once kappa is large."""
    a = _with_condition(kappa, cols=cols)
    start = slso.QR_AUTO if path == "auto" else slso.QR_PANEL
    r, used = ctx.qr_r_path(dev(a.copy()), start)
    r = host(r)
    want = {"cholqr2": {slso.QR_CHOLQR2}, "cholqr2_full": {slso.QR_CHOLQR2_FULL},
            "panel": {slso.QR_PANEL},
            "panel_or_tree": {slso.QR_PANEL, slso.QR_TREE}}[expect]
    assert used in want, used
    assert np.all(np.isfinite(r)) and np.all(np.diag(r) >= 0)
    g = a.T @ a
    err = np.abs(r.T @ r - g).max() / np.abs(g).max()
    print(f"[qr kappa={kappa:.0e} {path}] path {used} backward err {err:.2e}",
          flush=True)
    assert err < 1e-13


def test_qr_r_rank_deficient_falls_back(slso, ctx):
    """A zero column inside a 64-column panel makes both Cholesky-QR2 forms
    fail; the factorisation is redone column by column and stays a valid R."""
    a = np.random.default_rng(2).standard_normal((2000, 150))
    a[:, 70] = 0.0
    a[:, 20] = a[:, 3]          # a repeated column as well
    r, used = ctx.qr_r_path(dev(a.copy()))
    r = host(r)
    assert used == slso.QR_TREE
    assert np.all(np.isfinite(r))
    g = a.T @ a
    assert np.abs(r.T @ r - g).max() < 1e-12 * np.abs(g).max()
    assert abs(r[70, 70]) < 1e-12 * np.abs(r).max()


def test_qr_r_zero_column_is_finite(slso, ctx):
    a = np.random.default_rng(1).standard_normal((600, 40))
    a[:, 7] = 0.0
    r = host(ctx.qr_r(dev(a.copy())))
    assert np.all(np.isfinite(r))
    # past a zero column R is not unique; R^T R = A^T A is
    g = a.T @ a
    assert np.abs(r.T @ r - g).max() < 1e-12 * np.abs(g).max()
    assert r[7, 7] == 0.0


def test_qr_r_path_rejects_unknown(slso, ctx):
    with pytest.raises(slso.SlsoError) as e:
        ctx.qr_r_path(dev(np.zeros((8, 4))), 7)
    assert e.value.status == slso.EINVAL


# ---- triangular solve ------------------------------------------------------------
@pytest.mark.parametrize("d,k", [(1, 1), (63, 32), (64, 64), (65, 7), (200, 100)])
def test_solve_upper(slso, ctx, d, k):
    rng = np.random.default_rng(d + k)
    r = np.triu(rng.standard_normal((d, d))) + 4 * np.eye(d)
    b = rng.standard_normal((d, k))
    x = host(ctx.solve_upper(dev(r), dev(b.copy())))
    ref = sla.solve_triangular(r, b)
    assert np.abs(x - ref).max() / np.abs(ref).max() < 1e-12


# ---- scores ----------------------------------------------------------------------
@pytest.mark.parametrize("dtype,k", [("f64", 32), ("f32", 64), ("f32", 200),
                                     ("bf16", 16), ("f32", 1), ("f32", 37),
                                     ("bf16", 64), ("fp8", 64), ("bf16", 65)])
def test_scores_dense(slso, ctx, dtype, k):
    """k <= 64 with FP32, BF16 or FP8 input runs the MFMA kernel (ragged n
    and d); the others the FMA kernel. FP32 / BF16 / FP8 sums are FP32 within
    32-column chunks and FP64 across them; M enters BF16 MFMA as two BF16
    halves (relative error <= 2^-16 per element)."""
    rng = np.random.default_rng(k)
    n, d = 5003, 97
    x64 = rng.standard_normal((n, d))
    m = rng.standard_normal((d, k)) / np.sqrt(d)
    if dtype == "f64":
        xt, xref, tol = dev(x64), x64, 1e-7
    elif dtype == "f32":
        x32 = x64.astype(np.float32)
        xt, xref, tol = dev(x32), x32.astype(np.float64), 1e-5
    elif dtype == "bf16":
        bits = synth.to_bf16_bits(x64)
        xt = dev(bits.view(np.int16)).view(torch.bfloat16)
        xref, tol = synth.bf16_bits_to_f64(bits), 1e-5
    else:
        codes, cs = synth.to_fp8_e4m3(x64)
        xt = slso.Fp8Matrix(dev(codes), dev(cs))
        xref, tol = synth.fp8_e4m3_to_f64(codes, cs), 1e-5
    got = host(ctx.scores(xt, dev(m)))
    ref = olv.row_scores(xref, m)
    err = omet.max_rel_err(got, ref)
    print(f"[scores {dtype} k={k}] max_rel={err:.2e}", flush=True)
    if k >= 16:
        assert err < tol
    else:
        # few columns: a score can cancel to nearly nothing, so the rounding
        # of the sums is bounded by the sums of absolute values instead
        bound = ((np.abs(xref) @ np.abs(m)) ** 2).sum(axis=1)
        assert np.all(np.abs(got - ref) <= tol * bound)


def _fp8_every_code(ncols):
    """254 rows: every finite e4m3fn code once per column (rotated)."""
    finite = np.array([c for c in range(256) if (c & 0x7F) != 0x7F],
                      dtype=np.uint8)
    return np.stack([np.roll(finite, 17 * j) for j in range(ncols)], axis=1)


def test_fp8_every_code_countsketch_bit_exact(slso, ctx):
    """Every finite e4m3fn code in each of 16 columns with unit column
    scales: the decoded values are multiples of 2^-9 below 2^9, so the
    CountSketch's FP64 sums are exact and equal the oracle's bit for bit
    (pins the packed FP8 conversion of the CountSketch loads)."""
    codes = _fp8_every_code(16)
    cs = np.ones(16, np.float32)
    sx = host(ctx.sketch(slso.Fp8Matrix(dev(codes), dev(cs)), 3, 64))
    ref = osk.countsketch_dense(synth.fp8_e4m3_to_f64(codes, cs), 3, 64)
    assert np.array_equal(sx, ref)


@pytest.mark.parametrize("j", [0, 5, 15])
def test_fp8_every_code_scores_exact(slso, ctx, j):
    """The MFMA scoring path of FP8 input (d = 16, k = 1, M = e_j): l_i =
    x_ij^2, exact in FP32 (four significant bits squared), for every finite
    code (pins the packed FP8 conversion of the MFMA operands)."""
    codes = _fp8_every_code(16)
    cs = np.ones(16, np.float32)
    m = np.zeros((16, 1))
    m[j, 0] = 1.0
    got = host(ctx.scores(slso.Fp8Matrix(dev(codes), dev(cs)), dev(m)))
    xref = synth.fp8_e4m3_to_f64(codes, cs)
    assert np.array_equal(got.astype(np.float64), xref[:, j] ** 2)


@pytest.mark.parametrize("dtype,n,d,k", [
    ("bf16", 4099, 512, 64), ("bf16", 31, 16, 1), ("bf16", 70001, 496, 37),
    ("fp8", 5003, 512, 64), ("fp8", 1000, 272, 64), ("bf16", 300, 64, 64),
    ("bf16", 20011, 352, 32), ("bf16", 3000, 368, 64)])
def test_scores_m_in_lds(slso, ctx, dtype, n, d, k):
    """BF16 / FP8 input with d a multiple of 16 up to 512 and k <= 64: M
    enters the MFMA as BF16 parts held in LDS, X straight from HBM into the
    operands (ragged n, more blocks than waves). Three parts (M to FP32
    precision) up to d = 352: the FP32 bar, 1e-5 relative for k >= 16; two
    parts above (M to 2^-17 per entry) and FP32 sums of d exact products:
    |l - l_ref| <= 1e-4 sum_c (sum_j |x_ij M_jc|)^2."""
    rng = np.random.default_rng(n + d)
    x64 = rng.standard_normal((n, d)) * np.exp(rng.standard_normal(n))[:, None]
    m = rng.standard_normal((d, k)) / np.sqrt(d)
    if dtype == "bf16":
        bits = synth.to_bf16_bits(x64)
        xt = dev(bits.view(np.int16)).view(torch.bfloat16)
        xref = synth.bf16_bits_to_f64(bits)
    else:
        codes, cs = synth.to_fp8_e4m3(x64)
        xt = slso.Fp8Matrix(dev(codes), dev(cs))
        xref = synth.fp8_e4m3_to_f64(codes, cs)
    got = host(ctx.scores(xt, dev(m)))
    ref = olv.row_scores(xref, m)
    bound = ((np.abs(xref) @ np.abs(m)) ** 2).sum(axis=1)
    print(f"[scores lds {dtype} n={n} d={d} k={k}] max_rel="
          f"{omet.max_rel_err(got, ref):.2e} max err/bound="
          f"{(np.abs(got - ref) / bound).max():.2e}", flush=True)
    assert np.all(np.abs(got - ref) <= 1e-4 * bound)
    if d <= 352 and k >= 16:
        assert omet.max_rel_err(got, ref) < 1e-5


def test_scores_csr(slso, ctx):
    c = synth.text_like_csr(20000, 700, density=0.02, seed=4)
    m = np.random.default_rng(2).standard_normal((700, 64)) / 8
    got = host(ctx.scores(csr_dev(slso, c), dev(m)))
    ref = olv.row_scores(c, m)
    assert omet.max_rel_err(got, ref) < 1e-6


@pytest.mark.parametrize("k", [1, 64, 100])
def test_scores_csr_long_and_empty_rows(slso, ctx, k):
    """CSR rows of 0 to 500 entries (several groups of 64 per row) and k
    over one or two groups of 64 columns: each score is a sum of FP64
    products of the FP32 entries and M in FP32, so the error is M's rounding
    to FP32: |l - l_ref| <= 1e-6 sum_c (sum_j |x_ij M_jc|)^2 (a single
    column can cancel, so relative error is bounded only for k >= 16);
    empty rows score exactly zero."""
    n, d = 3000, 500
    rng = np.random.default_rng(k)
    lengths = rng.choice([0, 1, 63, 64, 65, 128, 300, 500], size=n)
    c = _csr_rows(n, d, lengths, seed=k + 7)
    m = rng.standard_normal((d, k)) / np.sqrt(d)
    got = host(ctx.scores(csr_dev(slso, c), dev(m)))
    ref = olv.row_scores(c, m)
    empty = np.diff(c.row_ptr) == 0
    assert np.all(got[empty] == 0.0)
    bound = ((np.abs(c.to_dense()) @ np.abs(m)) ** 2).sum(axis=1)
    assert np.all(np.abs(got - ref) <= 1e-6 * bound)
    if k >= 16:
        assert omet.max_rel_err(got[~empty], ref[~empty]) < 1e-6


# ---- sampling policies (Algorithm 4 step 4) ---------------------------------------
@pytest.mark.parametrize("n", [1, 2, 3000, 65537])
@pytest.mark.parametrize("epoch", [0, 7])
def test_order_swr_swor_match_oracle(slso, ctx, n, epoch):
    rng = np.random.default_rng(n + epoch)
    s = rng.random(n).astype(np.float32) ** 3
    if n > 10:
        s[rng.integers(0, n, n // 20)] = 0.0      # probability 0
        s[rng.integers(0, n, n // 50)] = -1.0     # probability 0
        s[rng.integers(0, n, n // 20)] = np.float32(0.125)   # ties
    sd = dev(s)
    swr = host(ctx.order_sample(sd, slso.ORDER_SWR, 99, epoch)).astype(np.int64)
    assert np.array_equal(swr, oorder.swr_order(s, 99, epoch))
    swor = host(ctx.order_sample(sd, slso.ORDER_SWOR, 99, epoch)).astype(np.int64)
    assert np.array_equal(swor, oorder.swor_order(s, 99, epoch))
    dec = host(ctx.order_sample(sd, slso.ORDER_DEC, 99, epoch)).astype(np.int64)
    assert np.array_equal(dec, np.argsort(-s, kind="stable"))


def test_order_sampling_special_cases(slso, ctx):
    z = dev(np.zeros(1000, np.float32))
    with pytest.raises(slso.SlsoError) as ei:
        ctx.order_sample(z, slso.ORDER_SWR, 1, 0)
    assert ei.value.status == slso.EINVAL
    # without replacement, all-zero scores keep the row order
    assert np.array_equal(host(ctx.order_sample(z, slso.ORDER_SWOR, 1, 0)),
                          np.arange(1000))
    with pytest.raises(slso.SlsoError):
        ctx.order_sample(z, 5, 1, 0)
    one = np.zeros(5000, np.float32)
    one[1234] = 3.0
    assert np.all(host(ctx.order_sample(dev(one), slso.ORDER_SWR, 2, 3)) == 1234)


def test_order_sampling_large_and_epochs_differ(slso, ctx):
    """Bench-sized scores (n = 60000) and a larger n spanning many scan
    blocks; successive epochs give different draws."""
    for n in (60000, 300001):
        s = (np.random.default_rng(n).random(n).astype(np.float32) + 0.01) ** 4
        sd = dev(s)
        a = host(ctx.order_sample(sd, slso.ORDER_SWR, 5, 0)).astype(np.int64)
        b = host(ctx.order_sample(sd, slso.ORDER_SWR, 5, 1)).astype(np.int64)
        assert not np.array_equal(a, b)
        if n == 60000:
            assert np.array_equal(a, oorder.swr_order(s, 5, 0))
            assert np.array_equal(
                host(ctx.order_sample(sd, slso.ORDER_SWOR, 5, 2)).astype(np.int64),
                oorder.swor_order(s, 5, 2))
        else:
            # frequencies follow P (chi-square over 40 equal-mass bins)
            cum = np.cumsum(s.astype(np.float64))
            edges = np.searchsorted(cum, cum[-1] * np.arange(1, 40) / 40)
            counts = np.bincount(np.searchsorted(edges, a, side="right"),
                                 minlength=40)
            from scipy import stats
            assert stats.chisquare(counts).pvalue > 1e-4
