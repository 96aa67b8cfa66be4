"""GPU tests of the leverage job enqueued with every decision on the device
(SLSO_OPT_NO_SYNC + slso_leverage_finish), through the C ABI.

The device path runs the same kernels as the synchronous one; the host
decisions (second Cholesky-QR pass, the form of R^{-1}, the rank screen)
become exit flags the kernels read. Its scores must therefore equal the
synchronous call's bit for bit, and its info (flags, diag(R) extremes) must
be the same. A job the device path leaves to the host (rank deficient, so
truncated) is rerun by slso_leverage_finish and then equals the synchronous
call too. The whole job is one enqueue with no host wait, so it can be
captured in a HIP graph: each replay, with new data written into the
captured input in between, must equal the eager call on that data.
"""
import numpy as np
import pytest

import synth
from oracle import leverage as olv
from oracle import metrics as omet

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


def _bf16(x64):
    return dev(synth.to_bf16_bits(x64).view(np.int16)).view(torch.bfloat16)


def _csr(slso, c):
    return slso.CsrMatrix(c.n, c.d, dev(c.row_ptr.astype(np.int64)),
                          dev(c.col_idx.astype(np.int32)),
                          dev(c.val.astype(np.float32)))


def _spread(n, d, kappa, seed):
    rng = np.random.default_rng(seed)
    u, _ = np.linalg.qr(rng.standard_normal((n, d)))
    v, _ = np.linalg.qr(rng.standard_normal((d, d)))
    return (u * np.logspace(0, -np.log10(kappa), d)) @ v.T


def _case(slso, name):
    """(input, seed, r, k, leverage keyword arguments) of one workload."""
    if name == "f64 countsketch":
        return dev(synth.config0()), 2000, 4096, 32, {}
    if name == "f32 countsketch fused":
        return dev(synth.image_like(20011, 200, seed=3)), 5, 2048, 64, {}
    if name == "f32 countsketch d1024":
        x = synth.lowrank_dense(60000, 1024, 512,
                                2.0 ** (-np.arange(512) / 4.0), 1e-3, 1.0,
                                seed=31).astype(np.float32)
        return dev(x), 6, 8192, 64, {}
    if name == "bf16 gaussian":
        return (_bf16(synth.config0(n=30001, d=64, seed=4)), 8, 512, 32,
                {"sketch": slso.GAUSSIAN})
    if name == "f32 gaussian":
        return (dev(synth.config0(n=20000, d=64, seed=9).astype(np.float32)),
                8, 512, 32, {"sketch": slso.GAUSSIAN})
    if name == "fp8 gaussian":
        codes, cs = synth.to_fp8_e4m3(synth.config0(n=20000, d=96, seed=12))
        return (slso.Fp8Matrix(dev(codes), dev(cs)), 13, 768, 32,
                {"sketch": slso.GAUSSIAN})
    if name == "f64 srht":
        return dev(synth.config0(n=5000, d=40, seed=2)), 33, 512, 16, \
            {"sketch": slso.SRHT}
    if name == "f32 osnap":
        return (dev(synth.image_like(9000, 130, seed=4)), 14, 1024, 17,
                {"sketch": slso.OSNAP, "nnz": 4})
    if name == "csr countsketch":
        return _csr(slso, synth.text_like_csr(30000, 800, seed=6)), 9, 4096, \
            64, {}
    if name.startswith("kappa"):
        # 2 r d^2 >= 2^31: the one-pass test is tried
        kappa = float(name.split()[1])
        return dev(_spread(30000, 576, kappa, int(kappa))), 11, 4096, 32, {}
    raise ValueError(name)


CASES = ["f64 countsketch", "f32 countsketch fused", "f32 countsketch d1024",
         "bf16 gaussian", "f32 gaussian", "fp8 gaussian", "f64 srht",
         "f32 osnap", "csr countsketch", "kappa 30", "kappa 3e3",
         "kappa 1e6"]


def _same_info(a, b):
    for key in ("status", "rank", "screen_full", "flags"):
        assert a[key] == b[key], (key, a, b)
    assert a["diag_min"] == b["diag_min"] and a["diag_max"] == b["diag_max"]


@pytest.mark.parametrize("name", CASES)
def test_no_sync_equals_sync(slso, ctx, name):
    x, seed, r, k, kw = _case(slso, name)
    ref, info = ctx.leverage(x, seed, r, k, **kw)
    ref = host(ref).copy()
    out, none = ctx.leverage(x, seed, r, k, no_sync=True, **kw)
    assert none is None
    info2 = ctx.leverage_finish()
    got = host(out)
    print(f"[no-sync {name}] flags={info2['flags']} rank={info2['rank']}",
          flush=True)
    assert not info2["flags"] & slso.INFO_RERUN
    _same_info(info2, info)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_no_sync_second_pass_and_one_pass_taken(slso, ctx):
    """The device decisions cover the three Cholesky-QR outcomes: one pass
    (kappa 30), two passes with the near-identity correction (kappa 3e3),
    and the second Cholesky (kappa 1e6)."""
    want = {"kappa 30": slso.INFO_QR_ONE_PASS, "kappa 3e3": 0,
            "kappa 1e6": slso.INFO_QR_SECOND_CHOLESKY}
    for name, bit in want.items():
        x, seed, r, k, kw = _case(slso, name)
        ctx.leverage(x, seed, r, k, no_sync=True, **kw)
        info = ctx.leverage_finish()
        mask = slso.INFO_QR_ONE_PASS | slso.INFO_QR_SECOND_CHOLESKY
        assert info["flags"] & mask == bit, (name, info)


def test_no_sync_rank_deficient_is_rerun(slso, ctx):
    """Noise-free rank-16 input in d = 32: the device rank screen trips, the
    job is rerun on the synchronous path (truncation), and the result equals
    the synchronous call's and the oracle's."""
    rng = np.random.default_rng(16)
    n, d, k = 4000, 32, 16
    u = synth.haar(rng, n, k)
    x64 = (u * np.exp(rng.standard_normal(n))[:, None]) @ rng.standard_normal((k, d))
    x = dev(x64)
    ref, info = ctx.leverage(x, 4, 1024, 0)
    ref = host(ref).copy()
    out, _ = ctx.leverage(x, 4, 1024, 0, no_sync=True)
    info2 = ctx.leverage_finish()
    got = host(out)
    assert info2["flags"] & slso.INFO_RERUN
    assert info2["rank"] == info["rank"] == k
    assert info2["status"] == slso.RANK_DEFICIENT
    assert info2["flags"] & ~slso.INFO_RERUN == info["flags"]
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    orc = olv.sketched_leverage(x64, 4, 1024, 0)
    assert omet.max_rel_err(got, orc["scores"]) < 1e-5


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_no_sync_nonfinite_reported_by_finish(slso, ctx, dtype):
    x = synth.config0(n=3000, d=24, seed=1)
    x[17, 3] = np.nan
    xd = dev(x if dtype == "f64" else x.astype(np.float32))
    ctx.leverage(xd, 1, 256, 4, no_sync=True)
    with pytest.raises(slso.SlsoError) as ei:
        ctx.leverage_finish()
    assert ei.value.status == slso.ENONFINITE


def test_finish_without_a_call_rejected(slso):
    c = slso.Context(0)
    with pytest.raises(slso.SlsoError) as ei:
        c.leverage_finish()
    assert ei.value.status == slso.EINVAL
    c.close()


@pytest.mark.parametrize("name", ["f32 countsketch fused", "bf16 gaussian"])
def test_no_sync_graph_replays(slso, name):
    """The job captured once in a HIP graph (torch.cuda.graph) and replayed
    four times; before each replay new data is copied into the captured
    input with eager work on the device; each replay must equal the eager
    synchronous call on that data, bit for bit."""
    ctx = slso.Context(0)
    x, seed, r, k, kw = _case(slso, name)
    datas = []
    for rep in range(4):
        if name.startswith("bf16"):
            xi = _bf16(synth.config0(n=x.shape[0], d=x.shape[1], seed=50 + rep))
        else:
            xi = dev(synth.image_like(x.shape[0], x.shape[1],
                                      seed=50 + rep).astype(np.float32))
        datas.append(xi)
    # the workspace is grown by an eager call of this size before capture
    ctx.leverage(x, seed, r, k, no_sync=True, **kw)
    ctx.leverage_finish()
    refs = []
    for xi in datas:
        sc, info = ctx.leverage(xi, seed, r, k, **kw)
        refs.append((host(sc).copy(), info))
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        out, _ = ctx.leverage(x, seed, r, k, no_sync=True, **kw)
    torch.cuda.synchronize()
    for rep, xi in enumerate(datas):
        x.copy_(xi)
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between
        g.replay()
        torch.cuda.synchronize()
        info = ctx.leverage_finish()
        got = out.cpu().numpy()
        assert float(junk) == float(junk)
        assert not info["flags"] & slso.INFO_RERUN, (rep, info)
        _same_info(info, refs[rep][1])
        assert np.array_equal(got.view(np.uint32),
                              refs[rep][0].view(np.uint32)), rep
    del g
    ctx.close()
