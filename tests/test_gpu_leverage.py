"""End-to-end GPU parity of slso_leverage / slso_order against the oracle's
sketched leverage (same seed, hash, sign and Pi_2 streams), at the sizes of
the paper-shaped workloads. Tolerance: the FP32 gate, max relative score
error <= 1e-5 against the FP64 oracle; permutations bit-exact against a
stable descending sort of the GPU's own scores."""
import time

import numpy as np
import pytest

import synth
from oracle import leverage as olv
from oracle import metrics as omet
from oracle import sketch as osk

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
    tau = omet.kendall_tau(got, ref)
    print(f"[{name}] max_rel={err:.3e} kendall_tau={tau:.6f} {extra}", flush=True)
    return err, tau


def test_config0_full(slso, ctx):
    """n=20000, d=64, FP64, CountSketch r=4096, k=32 (plain-method workload)."""
    x = synth.config0()
    seed = 2000
    got, info = ctx.leverage(dev(x), seed, 4096, 32)
    got = host(got)
    ref = olv.sketched_leverage(x, seed, 4096, 32)
    assert info["rank"] == 64 and info["screen_full"]
    # 2 r d^2 = 3.4e7 flop, far below 2^31: the condition estimate would cost
    # more than the second Cholesky-QR pass, so both passes run
    assert not info["flags"] & slso.INFO_QR_ONE_PASS
    err, _ = _report("c0", got, ref["scores"])
    assert err < 1e-5
    exact, _ = olv.exact_leverage(x)
    _report("c0 vs exact (context)", got, exact)
    perm = host(ctx.order(dev(got))).astype(np.int64)
    assert np.array_equal(perm, np.argsort(-got, kind="stable"))


@pytest.mark.parametrize("kappa,one", [(30.0, True), (3e3, False), (1e6, False)])
def test_one_pass_taken_only_when_its_bound_holds(slso, ctx, kappa, one):
    """FP64 X (n = 30000, d = 576, r = 4096: 2 r d^2 = 2.7e9 >= 2^31, so the
    one-pass test is tried) with singular values spread over kappa: one
    Cholesky-QR pass exactly when 4 kappa_est^2 sqrt(r d) 2^-53 <= 1e-7
    (kappa 30: about 6e-10; 3e3: 6e-6; 1e6: 0.6), and the scores within the
    FP32 gate either way (FP64 input, so well inside it)."""
    rng = np.random.default_rng(int(kappa))
    n, d, r = 30000, 576, 4096
    u, _ = np.linalg.qr(rng.standard_normal((n, d)))
    v, _ = np.linalg.qr(rng.standard_normal((d, d)))
    x = (u * np.logspace(0, -np.log10(kappa), d)) @ v.T
    got, info = ctx.leverage(dev(x), 11, r, 32)
    got = host(got)
    ref = olv.sketched_leverage(x, 11, r, 32)
    err, _ = _report(f"one pass kappa={kappa:g} flags={info['flags']}", got,
                     ref["scores"])
    assert bool(info["flags"] & slso.INFO_QR_ONE_PASS) == one
    assert err < (1e-6 if one else 1e-5)


def test_config0_k0_exact_sketched_scores(slso, ctx):
    x = synth.config0(n=6000, d=40, seed=5)
    got, _ = ctx.leverage(dev(x), 7, 1024, 0)
    ref = olv.sketched_leverage(x, 7, 1024, 0)
    err, _ = _report("c0 k=0", host(got), ref["scores"])
    assert err < 1e-5


def test_config1_full(slso, ctx):
    """n=60000, d=784, FP32 in [0,1], CountSketch r=16384, k=64."""
    x = synth.config1()
    seed = 2001
    t0 = time.time()
    got, info = ctx.leverage(dev(x), seed, 16384, 64)
    got = host(got)
    t1 = time.time()
    ref = olv.sketched_leverage(x, seed, 16384, 64)
    t2 = time.time()
    assert info["rank"] == 784
    err, tau = _report("c1", got, ref["scores"],
                       f"gpu {t1 - t0:.2f}s oracle {t2 - t1:.2f}s")
    assert err < 1e-5
    assert tau > 0.999
    perm = host(ctx.order(dev(got))).astype(np.int64)
    assert np.array_equal(perm, np.argsort(-got, kind="stable"))


def test_config1_ragged_small(slso, ctx):
    x = synth.image_like(2999, 130, seed=8)
    got, _ = ctx.leverage(dev(x), 3, 1000, 17)
    ref = olv.sketched_leverage(x, 3, 1000, 17)
    err, _ = _report("c1 ragged", host(got), ref["scores"])
    assert err < 1e-5


@pytest.mark.parametrize("n,d", [(5000, 200), (4097, 196)])
def test_fp32_k64_scoring_forms(slso, ctx, n, d):
    """FP32 input with k = 64: d = 200 takes the split-BF16 scoring (d a
    multiple of 8; its last 32-column chunk is partial), d = 196 the FP32
    MFMA; both within the FP32 gate of the oracle."""
    x = synth.image_like(n, d, seed=60 + d)
    assert x.dtype == np.float32
    got, info = ctx.leverage(dev(x), 21, 2048, 64)
    ref = olv.sketched_leverage(x, 21, 2048, 64)
    assert info["rank"] == d
    err, tau = _report(f"fp32 k64 d={d}", host(got), ref["scores"])
    assert err < 1e-5
    assert tau > 0.999


@pytest.mark.parametrize("d,nnz", [(128, 2), (130, 4), (784, 2)])
def test_osnap_leverage(slso, ctx, d, nnz):
    """OSNAP sketch (nnz nonzeros per column of S), FP32 input: d = 128 and
    784 take the CountSketch pass with the column maxima, d = 130 (row stride
    not a multiple of 4) the two-pass path."""
    n, r = (60000, 16384) if d == 784 else (6000, 2048)
    x = synth.image_like(n, d, seed=d + nnz)
    got, info = ctx.leverage(dev(x), 31, r, 32, sketch=slso.OSNAP, nnz=nnz)
    ref = olv.sketched_leverage(x, 31, r, 32, kind="osnap", nnz=nnz)
    assert info["rank"] == ref["rank"]
    err, tau = _report(f"osnap d={d} s={nnz}", host(got), ref["scores"])
    assert err < 1e-5


@pytest.mark.parametrize("n,d,r", [(6000, 128, 2048), (60000, 784, 16384)])
def test_srht_leverage(slso, ctx, n, d, r):
    x = synth.image_like(n, d, seed=d + 1)
    got, info = ctx.leverage(dev(x), 33, r, 32, sketch=slso.SRHT)
    ref = olv.sketched_leverage(x, 33, r, 32, kind="srht")
    assert info["rank"] == ref["rank"]
    err, _ = _report(f"srht n={n} d={d}", host(got), ref["scores"])
    assert err < 1e-5


def test_osnap_csr_leverage(slso, ctx):
    c = synth.text_like_csr(30000, 800, seed=7)
    xc = slso.CsrMatrix(c.n, c.d, dev(c.row_ptr.astype(np.int64)),
                        dev(c.col_idx.astype(np.int32)),
                        dev(c.val.astype(np.float32)))
    got, info = ctx.leverage(xc, 12, 4096, 64, sketch=slso.OSNAP, nnz=2)
    ref = olv.sketched_leverage(c, 12, 4096, 64, kind="osnap", nnz=2)
    assert info["rank"] == ref["rank"]
    err, _ = _report("osnap csr", host(got), ref["scores"])
    assert err < 1e-5


def test_csr_small(slso, ctx):
    c = synth.text_like_csr(30000, 800, seed=6)
    xc = slso.CsrMatrix(c.n, c.d, dev(c.row_ptr.astype(np.int64)),
                        dev(c.col_idx.astype(np.int32)),
                        dev(c.val.astype(np.float32)))
    got, info = ctx.leverage(xc, 9, 4096, 64)
    ref = olv.sketched_leverage(c, 9, 4096, 64)
    assert info["rank"] == ref["rank"]
    err, _ = _report("csr small", host(got), ref["scores"])
    assert err < 1e-5


def test_rank_deficient_truncation(slso, ctx):
    """Noise-free rank-16 input in d=32: the screen trips, the Jacobi SVD finds
    rank 16, and the truncated scores match the oracle's; with truncation
    disabled the scores are far from the exact ones (Figs. 2-3 analog)."""
    rng = np.random.default_rng(16)
    n, d, k = 4000, 32, 16
    u = synth.haar(rng, n, k)
    x = (u * np.exp(rng.standard_normal(n))[:, None]) @ rng.standard_normal((k, d))
    got, info = ctx.leverage(dev(x), 4, 1024, 0)
    assert info["rank"] == k and not info["screen_full"]
    assert info["status"] == slso.RANK_DEFICIENT
    ref = olv.sketched_leverage(x, 4, 1024, 0)
    assert ref["rank"] == k
    err, _ = _report("rank-deficient", host(got), ref["scores"])
    assert err < 1e-5
    exact, _ = olv.exact_leverage(x)
    bad, info2 = ctx.leverage(dev(x), 4, 1024, 0, rank_tol=-1.0)
    bad = host(bad)
    assert info2["rank"] == d
    assert (not np.all(np.isfinite(bad))) or omet.max_rel_err(bad, exact) > 1.0


def test_nonfinite_input_rejected(slso, ctx):
    x = synth.config0(n=500, d=8, seed=1)
    x[17, 3] = np.nan
    with pytest.raises(slso.SlsoError) as ei:
        ctx.leverage(dev(x), 1, 64, 4)
    assert ei.value.status == slso.ENONFINITE


@pytest.mark.parametrize("bad", [np.nan, np.inf])
def test_nonfinite_fp32_rejected(slso, ctx, bad):
    """FP32 input: the column maxima come from the CountSketch's own pass."""
    x = synth.image_like(500, 64, seed=2)
    x[17, 3] = bad
    with pytest.raises(slso.SlsoError) as ei:
        ctx.leverage(dev(x), 1, 128, 4)
    assert ei.value.status == slso.ENONFINITE


def test_invalid_sizes_rejected(slso, ctx):
    x = synth.config0(n=500, d=8, seed=1)
    with pytest.raises(slso.SlsoError) as ei:
        ctx.leverage(dev(x), 1, 4, 4)      # r < d
    assert ei.value.status == slso.EINVAL
    with pytest.raises(slso.SlsoError):
        ctx.leverage(dev(x), 1, 64, -1)    # k < 0


# ---- sketched SVD and the SVD rank decision ----------------------------------------
@pytest.mark.parametrize("kind,n,d,r", [("countsketch", 4000, 40, 512),
                                        ("osnap", 3000, 64, 1024),
                                        ("countsketch", 20000, 200, 2048)])
def test_sketch_svd_matches_oracle(slso, ctx, kind, n, d, r):
    x = synth.config0(n=n, d=d, seed=d)
    sk = slso.OSNAP if kind == "osnap" else slso.COUNTSKETCH
    sig, v = ctx.sketch_svd(dev(x), 3, r, sketch=sk, nnz=2)
    sig, v = host(sig), host(v)
    rs, rv = olv.sketched_svd(x, 3, r, kind=kind, nnz=2)
    assert np.max(np.abs(sig - rs) / rs[0]) < 1e-12
    # right singular vectors (distinct singular values: sigma_j = 2^(-j/4))
    assert np.max(np.abs(v - rv)) < 1e-8
    sx = osk.countsketch_dense(x, 3, r) if kind == "countsketch" else \
        osk.osnap_dense(x, 3, r, 2)
    g = sx.T @ sx
    assert np.max(np.abs(v @ np.diag(sig ** 2) @ v.T - g)) < 1e-11 * sig[0] ** 2


def test_svd_rank_mode(slso, ctx):
    """A Kahan-type factor: X = Q K with Q orthonormal columns. The diagonal
    screen calls the sketch's R full rank; the SVD decision cuts its smallest
    singular value. Both modes match the oracle's."""
    rng = np.random.default_rng(60)
    d, c = 40, 0.3
    s_ = np.sqrt(1 - c * c)
    kahan = np.diag(s_ ** np.arange(d)) @ (np.triu(-c * np.ones((d, d)), 1) + np.eye(d))
    x = synth.haar(rng, 8000, d) @ kahan
    seed, r = 7, 1024
    base = olv.sketched_leverage(x, seed, r, 0)
    sv = np.linalg.svd(base["R_D"], compute_uv=False)
    tol = float(np.sqrt(sv[-1] * sv[-2]) / sv[0])   # between the last two
    dg = np.abs(np.diag(base["R_D"]))
    if not dg.min() > np.sqrt(tol) * dg.max():
        pytest.skip("this sketch's diagonal already trips the screen")
    ref_screen = olv.sketched_leverage(x, seed, r, 0, rank_tol=tol)
    ref_svd = olv.sketched_leverage(x, seed, r, 0, rank_tol=tol, always_svd=True)
    assert ref_screen["rank"] == d and ref_svd["rank"] == d - 1
    got, info = ctx.leverage(dev(x), seed, r, 0, rank_tol=tol)
    assert info["rank"] == d
    assert _report("kahan screen", host(got), ref_screen["scores"])[0] < 1e-5
    got2, info2 = ctx.leverage(dev(x), seed, r, 0, rank_tol=tol, svd_rank=True)
    assert info2["rank"] == d - 1 and not info2["screen_full"]
    assert _report("kahan svd rank", host(got2), ref_svd["scores"])[0] < 1e-5
    # full-rank input: the SVD decision keeps everything and gives R^{-1}'s scores
    y = synth.config0(n=6000, d=32, seed=61)
    a, ia = ctx.leverage(dev(y), 3, 1024, 16, svd_rank=True)
    ref = olv.sketched_leverage(y, 3, 1024, 16)
    assert ia["rank"] == 32
    assert _report("full rank, svd decision", host(a), ref["scores"])[0] < 1e-5


def test_calls_on_two_streams_share_the_workspace_in_order(slso, ctx):
    """Two leverage calls and their orderings issued back to back on two
    streams, with no synchronisation between them, use one context's
    workspace: the second call's sketch must not overwrite what the first
    call's scoring pass still reads. Each result must equal, bit for bit,
    the same call made alone."""
    n, d, r, k = 200003, 256, 2048, 64
    xs = [dev(synth.lowrank_dense(n, d, d // 2,
                                  2.0 ** (-np.arange(d // 2) / 4.0), 1e-3, 1.0,
                                  seed=300 + i).astype(np.float32))
          for i in range(2)]
    alone = []
    for i, x in enumerate(xs):
        sc, _ = ctx.leverage(x, 40 + i, r, k)
        pm = ctx.order(sc)
        alone.append((host(sc).copy(), host(pm).copy()))
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in xs]
    perms = [torch.empty(n, dtype=torch.int32, device="cuda") for _ in xs]
    torch.cuda.synchronize()
    for rep in range(3):
        for i, x in enumerate(xs):
            ctx.leverage(x, 40 + i, r, k, out=outs[i], stream=streams[i])
            ctx.order(outs[i], out=perms[i], stream=streams[i])
        torch.cuda.synchronize()
        for i in range(2):
            assert np.array_equal(host(outs[i]).view(np.uint32),
                                  alone[i][0].view(np.uint32)), (rep, i)
            assert np.array_equal(host(perms[i]), alone[i][1]), (rep, i)


@pytest.mark.parametrize("kind,sketch,refine,r,tol", [
    ("f32", "countsketch", False, 1024, 1e-8),
    ("f32", "countsketch", True, 1024, 1e-8),
    ("f32", "gaussian", False, 256, 1e-5),
    ("bf16", "gaussian", True, 512, 1e-4)])
def test_eps_hat_matches_oracle(slso, ctx, kind, sketch, refine, r, tol):
    """Realised distortion of the sketch on range(X) (Def. 1 / Thm. 1): the
    library's 1 / sigma(R1) route against the oracle's sigma(S U). FP32
    input: the Gram is exact (FP64 MFMA), and so is the CountSketch; the
    FP32 Gaussian sketch carries FP32 sums (about 1e-7 of each entry); BF16:
    FP32 sums of the Gram as well."""
    x64 = synth.config0(n=20011, d=48, seed=41)
    if kind == "f32":
        x32 = x64.astype(np.float32)
        xin, xval, prec = dev(x32), x32.astype(np.float64), "f32"
    else:
        b = synth.to_bf16_bits(x64)
        xin = dev(b.view(np.int16)).view(torch.bfloat16)
        xval, prec = synth.bf16_bits_to_f64(b), "bf16"
    sk = slso.GAUSSIAN if sketch == "gaussian" else slso.COUNTSKETCH
    got, info = ctx.leverage(xin, 17, r, 16, sketch=sk, refine=refine,
                             eps_hat=True)
    ref = olv.realised_distortion(xval, 17, r, kind=sketch, precision=prec)
    print(f"[eps_hat {kind} {sketch} refine={refine}] gpu={info['eps_hat']:.10f}"
          f" oracle={ref:.10f}", flush=True)
    assert abs(info["eps_hat"] - ref) <= tol * max(1.0, ref)
    # the report changes nothing else: same scores as without it
    base, _ = ctx.leverage(xin, 17, r, 16, sketch=sk, refine=refine)
    np.testing.assert_allclose(host(got), host(base), rtol=1e-6)


def test_fixed_workspace_context(slso):
    """A context created with a workspace size allocates it once: calls that
    fit give the same bits as on a context whose workspace grows, and a call
    that needs more fails with ENOMEM, enqueues nothing and leaves the
    context usable."""
    x = dev(synth.config0(n=20000, d=64, seed=3))
    need = slso.workspace_size(x, 4096, 32)
    auto = slso.Context(0)
    ref, _ = auto.leverage(x, 5, 4096, 32)
    pref = host(auto.order(ref)).copy()
    ref = host(ref).copy()
    auto.close()
    fixed = slso.Context(0, workspace_bytes=need)
    got, info = fixed.leverage(x, 5, 4096, 32)
    perm = host(fixed.order(got))
    assert info["rank"] == 64
    assert np.array_equal(host(got).view(np.uint32), ref.view(np.uint32))
    assert np.array_equal(perm, pref)
    big = dev(synth.config0(n=40000, d=128, seed=4))
    with pytest.raises(slso.SlsoError) as ei:
        fixed.leverage(big, 5, 8192, 32)
    assert ei.value.status == slso.ENOMEM
    again, _ = fixed.leverage(x, 5, 4096, 32)
    assert np.array_equal(host(again).view(np.uint32), ref.view(np.uint32))
    fixed.close()
