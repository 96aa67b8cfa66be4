"""slso_scores_noalloc (the scoring call that allocates nothing, for callers
that cannot allocate) against slso_scores on the same input, through the C
ABI: the two run the same kernels, so the scores must be bit-identical. Two
calls in a row, the second on a smaller input, so the second call runs on
the scratch the first one left behind. Algorithm 2 step 4 (l_i = ||x_i M||^2)."""
import numpy as np
import pytest

import synth

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


def make_input(slso, kind, n, d, seed):
    rng = np.random.default_rng(seed)
    x64 = rng.standard_normal((n, d)) * np.exp(rng.standard_normal(n))[:, None]
    if kind == "f32":
        return dev(x64.astype(np.float32))
    if kind == "bf16":
        return dev(synth.to_bf16_bits(x64).view(np.int16)).view(torch.bfloat16)
    if kind == "fp8":
        codes, cs = synth.to_fp8_e4m3(x64)
        return slso.Fp8Matrix(dev(codes), dev(cs))
    dense = np.where(rng.random((n, d)) < 0.05, x64, 0.0).astype(np.float32)
    rp = np.concatenate([[0], np.cumsum((dense != 0).sum(axis=1))])
    ci = np.nonzero(dense)[1].astype(np.int32)
    val = dense[dense != 0].astype(np.float32)
    return slso.CsrMatrix(n, d, dev(rp.astype(np.int64)), dev(ci), dev(val))


@pytest.mark.parametrize("kind,big,small,k", [
    ("bf16", (200003, 512), (70001, 256), 64),   # M in LDS, two then three parts
    ("fp8", (150001, 320), (4099, 64), 32),
    ("f32", (100003, 97), (5003, 33), 64),       # split-BF16 MFMA scoring
    ("f32", (20011, 40), (3001, 17), 80),        # k > 64: FP64 partial sums
    ("csr", (60001, 300), (7001, 120), 16),
])
def test_noalloc_matches_scores(slso, ctx, kind, big, small, k):
    outs = []
    for i, (n, d) in enumerate((big, small)):
        x = make_input(slso, kind, n, d, 1000 + i)
        m = dev(np.random.default_rng(7 + i).standard_normal((d, k)) / np.sqrt(d))
        print(f"[noalloc {kind} n={n} d={d} k={k}]", flush=True)
        got = ctx.scores(x, m, noalloc=True)
        outs.append((x, m, got))
    for x, m, got in outs:
        ref = ctx.scores(x, m)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        assert torch.isfinite(got).all()


def test_noalloc_rejects_oversize(slso, ctx):
    """Buffers past the 16 MiB scratch are refused before anything runs."""
    d, k = 20000, 64   # d FP64 factors + M in FP64 and FP32 + BF16 parts > 16 MiB
    x = dev(np.ones((1, d), np.float32))
    m = dev(np.ones((d, k)))
    with pytest.raises(slso.SlsoError, match="scratch"):
        ctx.scores(x, m, noalloc=True)
    # the context still works afterwards
    got = ctx.scores(dev(np.ones((3, 8), np.float32)), dev(np.ones((8, 2))),
                     noalloc=True)
    torch.cuda.synchronize()
    assert torch.equal(got.cpu(), torch.full((3,), 128.0))
