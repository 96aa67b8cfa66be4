"""GPU parity of the Gaussian sketch, the FP8 input path and the Cholesky-QR
refinement against the CPU oracle, through the C ABI (gfx950).

Tolerances:
* generator entries: bit-exact (the FP32 generator: both sides evaluate the
  same sequence of separately rounded FP32 operations; the quantile form:
  the same Philox halves and the same tables);
* Gaussian sketch: the GPU sums exact BF16 (or FP32) products in FP32 within
  slices of at most 65536 rows (FP32 input) or 2^18 rows (BF16, FP8) and in
  FP64 across slices; the oracle sums in FP64. The error bound used is 1e-4
  of sum_i |g_ji x_ic| / sqrt(r), about 13x the random-walk estimate
  sqrt(m / 16) 2^-24 for slices of m = 2^18 rows;
* refined scores: the spec bar for the reduced-precision path, max
  relative error <= 1e-2 and Kendall tau >= 0.99 against the FP64 oracle;
  observed errors are far smaller and are printed.
"""
import math

import numpy as np
import pytest

import synth
from oracle import leverage as olv
from oracle import metrics as omet
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


def _report(name, got, ref, extra=""):
    err = omet.max_rel_err(got, ref)
    print(f"[{name}] max_rel={err:.3e} {extra}", flush=True)
    return err


def as_input(slso, x64, kind):
    """(device input, FP64 values it stands for, oracle generator precision)."""
    if kind == "f32":
        x32 = x64.astype(np.float32)
        return dev(x32), x32.astype(np.float64), "f32"
    if kind == "bf16":
        b = synth.to_bf16_bits(x64)
        t = dev(b.view(np.int16)).view(torch.bfloat16)
        return t, synth.bf16_bits_to_f64(b), "bf16"
    if kind == "fp8":
        codes, cs = synth.to_fp8_e4m3(x64)
        return (slso.Fp8Matrix(dev(codes), dev(cs)),
                synth.fp8_e4m3_to_f64(codes, cs), "fp8")
    raise ValueError(kind)


# ---- generator -----------------------------------------------------------------
@pytest.mark.parametrize("seed,r,row0,n", [
    (0, 1, 0, 1), (11, 7, 0, 4099), (2025, 300, 3, 1001),
    (2**63 + 5, 33, 2**33 + 17, 517), (1003, 2048, 123457, 64)])
def test_gaussian_sketch_entries_bit_exact(slso, seed, r, row0, n):
    g = host(slso.gaussian_sketch_entries(seed, r, n, row0=row0))
    ref = ost.gaussian_sketch_matrix_f32(seed, r, n, row0=row0)
    assert g.dtype == np.float32
    assert np.array_equal(g.view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("seed,r,row0,n", [
    (0, 1, 0, 1), (11, 7, 0, 4099), (2025, 300, 3, 1001),
    (2**63 + 5, 33, 2**33 + 13, 517), (1003, 2048, 123457, 64)])
@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_gaussian_sketch_entries_q_bit_exact(slso, seed, r, row0, n, fmt):
    """Quantile-form entries (BF16 and e4m3 tables, Philox halves) against
    the oracle's, bit for bit."""
    dt = slso.BF16 if fmt == "bf16" else slso.FP8_E4M3
    g = host(slso.gaussian_sketch_entries_q(seed, dt, r, n, row0=row0))
    ref = ost.gaussian_sketch_matrix_q(seed, r, n, fmt, row0=row0)
    assert np.array_equal(g.astype(np.float64), ref)


# ---- sketch ----------------------------------------------------------------------
@pytest.mark.parametrize("kind,n,d,r", [
    ("f32", 3001, 40, 300), ("bf16", 3001, 40, 300), ("fp8", 2999, 37, 257),
    ("bf16", 66000, 33, 257), ("f32", 520, 300, 520), ("bf16", 300007, 72, 257),
    ("fp8", 70001, 520, 600), ("bf16", 5003, 1030, 1100)])
def test_gaussian_sketch_matches_oracle(slso, ctx, kind, n, d, r):
    rng = np.random.default_rng(n + d)
    x64 = rng.standard_normal((n, d)) * np.exp(rng.standard_normal(n))[:, None]
    xin, xval, prec = as_input(slso, x64, kind)
    sx = host(ctx.sketch(xin, 99, r, sketch=slso.GAUSSIAN))
    g = (ost.gaussian_sketch_matrix_f32(99, r, n) if prec == "f32"
         else ost.gaussian_sketch_matrix_q(99, r, n, prec)).astype(np.float64)
    ref = osk.gaussian_sketch_dense(xval, 99, r, g=g)
    bound = 1e-4 * (np.abs(g) @ np.abs(xval)) / math.sqrt(r)
    err = np.abs(sx - ref)
    print(f"[gsketch {kind} {n}x{d} r={r}] max err/bound = "
          f"{(err / bound).max():.3e}", flush=True)
    assert np.all(err <= bound)


def test_fp8_countsketch_matches_oracle(slso, ctx):
    x64 = synth.config0(n=5000, d=48, seed=5)
    xin, xval, _ = as_input(slso, x64, "fp8")
    sx = host(ctx.sketch(xin, 3, 1024))
    ref = osk.countsketch_dense(xval, 3, 1024)
    # per-bucket FP64 sums of codes, scaled once: rounding-level difference
    scale = osk.countsketch_dense(np.abs(xval), 3, 1024) + 1e-300
    assert np.max(np.abs(sx - ref) / scale) < 1e-14


# ---- leverage with the Gaussian sketch (no refinement) -------------------------
@pytest.mark.parametrize("kind,n", [("f32", 20000), ("bf16", 20000),
                                    ("f32", 140001)])
def test_gaussian_leverage_matches_sketched_oracle(slso, ctx, kind, n):
    """Unrefined Gaussian-sketch leverage. FP32 input is the plain FP32 path
    (FP32 entries of S on the FP32 MFMA): the FP32 gate, <= 1e-5 against
    the FP64 oracle of the same sketch, at one row split (n = 20000) and at
    three (n = 140001: FP32 sums within splits of at most 65536 rows, FP64
    across them). BF16 input: the reduced-precision gate."""
    x64 = synth.config0(n=n, d=64, seed=21)
    xin, xval, prec = as_input(slso, x64, kind)
    got, info = ctx.leverage(xin, 8, 512, 32, sketch=slso.GAUSSIAN)
    got = host(got)
    ref = olv.sketched_leverage(xval, 8, 512, 32, kind="gaussian",
                                precision=prec)
    assert info["rank"] == ref["rank"] == 64
    assert not info["refined"]
    err = _report(f"gauss lev {kind} n={n}", got, ref["scores"])
    if kind == "f32":
        assert err <= 1e-5
    else:
        assert err <= 1e-2 and omet.kendall_tau(got, ref["scores"]) >= 0.99


def test_fp8_countsketch_leverage(slso, ctx):
    x64 = synth.config0(n=20000, d=64, seed=22)
    xin, xval, _ = as_input(slso, x64, "fp8")
    got, info = ctx.leverage(xin, 4, 4096, 32)
    got = host(got)
    ref = olv.sketched_leverage(xval, 4, 4096, 32)
    assert info["rank"] == ref["rank"]
    assert _report("fp8 countsketch lev", got, ref["scores"]) < 1e-5


@pytest.mark.parametrize("kind,d,pad", [
    ("f32", 70, 2), ("bf16", 70, 2), ("fp8", 70, 2), ("f32", 64, 0),
    ("f32", 33, 3), ("fp8", 33, 0), ("f32", 514, 2), ("bf16", 1030, 2)])
def test_countsketch_leverage_strided_rows(slso, ctx, kind, d, pad):
    """Row stride d + pad: the CountSketch that takes the column maxima in the
    same pass (rows starting on 4-element boundaries, a partial last vector
    when d % 4 != 0, in each of its width forms: d = 70, 514 and 1030) and,
    for a row stride of 33, the two-pass path."""
    x64 = synth.config0(n=3001, d=d, seed=23)
    xin, xval, _ = as_input(slso, np.pad(x64, ((0, 0), (0, pad))), kind)
    xval = xval[:, :d]
    if kind == "fp8":
        xin = slso.Fp8Matrix(xin.codes[:, :d], xin.col_scale[:d])
    else:
        xin = xin[:, :d]
    r = 1024 if d < 512 else 2 * d
    got, info = ctx.leverage(xin, 6, r, 32)
    got = host(got)
    ref = olv.sketched_leverage(xval, 6, r, 32)
    assert info["rank"] == ref["rank"]
    assert _report(f"countsketch lev {kind} d={d} ld={d + pad}", got,
                   ref["scores"]) < 1e-5


@pytest.mark.parametrize("kind", ["bf16", "fp8"])
def test_osnap_leverage_reduced_precision(slso, ctx, kind):
    x64 = synth.config0(n=20000, d=64, seed=24)
    xin, xval, _ = as_input(slso, x64, kind)
    got, info = ctx.leverage(xin, 5, 4096, 32, sketch=slso.OSNAP, nnz=4)
    ref = olv.sketched_leverage(xval, 5, 4096, 32, kind="osnap", nnz=4)
    assert info["rank"] == ref["rank"]
    assert _report(f"osnap lev {kind}", host(got), ref["scores"]) < 1e-5


@pytest.mark.parametrize("kind", ["bf16", "fp8"])
def test_srht_leverage_reduced_precision(slso, ctx, kind):
    x64 = synth.config0(n=20000, d=64, seed=25)
    xin, xval, _ = as_input(slso, x64, kind)
    got, info = ctx.leverage(xin, 6, 4096, 32, sketch=slso.SRHT)
    ref = olv.sketched_leverage(xval, 6, 4096, 32, kind="srht")
    assert info["rank"] == ref["rank"]
    assert _report(f"srht lev {kind}", host(got), ref["scores"]) < 1e-5


# ---- refinement ---------------------------------------------------------------------
@pytest.fixture(scope="module")
def precision_case():
    """Reduced-size precision workload (rank 256 in d = 512, sigma_j = j^-1.5,
    noise 1e-4, row scales e^N(0, 1.5^2)) with n = 100000."""
    return synth.precision_dense(n=100000, d=512, seed=1003)


@pytest.mark.parametrize("kind,sketch,k", [
    ("bf16", "gaussian", 64), ("fp8", "gaussian", 64), ("f32", "gaussian", 0),
    ("bf16", "countsketch", 64)])
def test_refined_leverage_vs_fp64_oracle(slso, ctx, precision_case, kind,
                                         sketch, k):
    xin, xval, _ = as_input(slso, precision_case, kind)
    sk = slso.GAUSSIAN if sketch == "gaussian" else slso.COUNTSKETCH
    r = 2048 if sketch == "gaussian" else 8192
    got, info = ctx.leverage(xin, 31, r, k, sketch=sk, refine=True)
    got = host(got)
    assert info["refined"], info
    ref = olv.sketched_leverage(xval, 31, r, k, refine=True)
    err = omet.max_rel_err(got, ref["scores"])
    tau = omet.kendall_tau(got, ref["scores"])
    print(f"[refined {kind} {sketch} k={k}] max_rel={err:.3e} tau={tau:.6f}",
          flush=True)
    assert info["rank"] == ref["rank"]
    assert err <= 1e-2 and tau >= 0.99


def test_refined_countsketch_f32_image_like(slso, ctx):
    x = synth.image_like(20000, 784, seed=44).astype(np.float32)
    got, info = ctx.leverage(dev(x), 6, 16384, 64, refine=True)
    got = host(got)
    ref = olv.sketched_leverage(x.astype(np.float64), 6, 16384, 64,
                                refine=True)
    assert info["refined"]
    err = _report("refined image-like f32", got, ref["scores"])
    assert err <= 1e-2 and omet.kendall_tau(got, ref["scores"]) >= 0.99


def test_refine_falls_back_on_rank_deficient_input(slso, ctx):
    """A zero column makes X D rank deficient: the refinement reports failure
    and the sketch factor with its truncation is used, so the scores equal
    those of the unrefined call."""
    rng = np.random.default_rng(9)
    x = rng.standard_normal((6000, 40)).astype(np.float32)
    x[:, 17] = 0.0
    xt = dev(x)
    got, info = ctx.leverage(xt, 2, 512, 16, sketch=slso.GAUSSIAN, refine=True)
    base, binfo = ctx.leverage(xt, 2, 512, 16, sketch=slso.GAUSSIAN)
    assert info["flags"] & slso.INFO_REFINE_FAILED
    # the zero column makes the sketch rank deficient as well: Cholesky-QR2
    # does not apply and its R comes from a Householder path
    assert info["flags"] & slso.INFO_QR_HOUSEHOLDER
    assert info["rank"] == binfo["rank"] == 39
    assert np.array_equal(host(got), host(base))


def test_gaussian_rejects_unsupported_inputs(slso, ctx):
    x = dev(np.zeros((100, 4)))
    with pytest.raises(slso.SlsoError) as e:
        ctx.leverage(x, 1, 16, 4, sketch=slso.GAUSSIAN)
    assert e.value.status == slso.EUNSUPPORTED
    with pytest.raises(slso.SlsoError) as e:
        ctx.leverage(x, 1, 16, 4, refine=True)
    assert e.value.status == slso.EUNSUPPORTED


@pytest.mark.parametrize("kind,bad,row,n", [
    ("bf16", np.nan, 17, 5000), ("bf16", np.inf, 4999, 5000),
    ("bf16", -np.inf, 70000, 100003), ("fp8", np.nan, 33, 5000)])
def test_gaussian_nonfinite_rejected(slso, ctx, kind, bad, row, n):
    """BF16 / FP8 input: the column maxima (and the Inf / NaN check) come from
    the Gaussian sketch's own pass, shared by its row-tile workgroups; a bad
    value in any row of any slice must be caught."""
    x64 = synth.config0(n=n, d=40, seed=3)
    xin, _, _ = as_input(slso, x64, kind)
    if kind == "fp8":
        xin.codes[row, 5] = 0x7F          # the e4m3fn NaN code
    else:
        xin[row, 5] = float(bad)
    with pytest.raises(slso.SlsoError) as ei:
        ctx.leverage(xin, 1, 512, 8, sketch=slso.GAUSSIAN)
    assert ei.value.status == slso.ENONFINITE


@pytest.mark.parametrize("kind,d,pad", [("bf16", 72, 0), ("bf16", 70, 3),
                                        ("fp8", 520, 0), ("fp8", 33, 5)])
def test_gaussian_equilibration_matches_oracle(slso, ctx, kind, d, pad):
    """Column scales D from the sketch pass (BF16, FP8; aligned rows and not)
    give the oracle's leverage: the unrefined Gaussian path against the
    sketched oracle of the same entries."""
    x64 = synth.config0(n=30011, d=d, seed=4)
    x64 *= np.exp(np.linspace(-6, 6, d))[None, :]   # columns over 2^17
    xin, xval, prec = as_input(slso, np.pad(x64, ((0, 0), (0, pad))), kind)
    xval = xval[:, :d]
    if kind == "fp8":
        xin = slso.Fp8Matrix(xin.codes[:, :d], xin.col_scale[:d])
    else:
        xin = xin[:, :d]
    r = 2 * d + 64
    got, info = ctx.leverage(xin, 12, r, 16, sketch=slso.GAUSSIAN)
    got = host(got)
    ref = olv.sketched_leverage(xval, 12, r, 16, kind="gaussian",
                                precision=prec)
    assert info["rank"] == ref["rank"]
    err = _report(f"gauss eq {kind} d={d} ld={d + pad}", got, ref["scores"])
    assert err <= 1e-2 and omet.kendall_tau(got, ref["scores"]) >= 0.99
