"""GPU tests of the tuned launch shapes (slso_tune, slso_tune_set), through
the C ABI: every choice of every tunable pass gives the same scores bit for
bit (the same sums in the same order), and slso_tune records a valid choice
for exactly the passes the input takes."""
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


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _input(slso, kind, n, d, seed):
    x64 = synth.config0(n=n, d=d, seed=seed)
    if kind == "f32":
        return dev(x64.astype(np.float32)), slso.F32
    if kind == "bf16":
        b = synth.to_bf16_bits(x64)
        return dev(b.view(np.int16)).view(torch.bfloat16), slso.BF16
    codes, cs = synth.to_fp8_e4m3(x64)
    return slso.Fp8Matrix(dev(codes), dev(cs)), slso.FP8_E4M3


CASES = [("bf16", 30001, 512, 2048, 64, "gaussian"),
         ("fp8", 30001, 352, 2048, 64, "gaussian"),
         ("bf16", 20011, 128, 1024, 32, "countsketch"),
         ("f32", 20011, 200, 2048, 64, "countsketch"),
         ("bf16", 20011, 600, 2048, 32, "countsketch"),
         ("f32", 9001, 1032, 2064, 32, "countsketch")]


@pytest.mark.parametrize("kind,n,d,r,k,sketch", CASES)
def test_tuned_shapes_give_identical_bits(slso, ctx, kind, n, d, r, k, sketch):
    x, dt = _input(slso, kind, n, d, seed=d)
    sk = slso.GAUSSIAN if sketch == "gaussian" else slso.COUNTSKETCH
    choices = {slso.TUNE_SCORE: 3, slso.TUNE_COUNTSKETCH: 2}
    for p in choices:
        slso.tune_set(p, d, dt, -1)
    ref, info = ctx.leverage(x, 5, r, k, sketch=sk)
    ref = host(ref).copy()
    for p, nc in choices.items():
        for ch in range(nc):
            slso.tune_set(p, d, dt, ch)
            got, _ = ctx.leverage(x, 5, r, k, sketch=sk)
            assert np.array_equal(host(got).view(np.uint32),
                                  ref.view(np.uint32)), (p, ch)
        slso.tune_set(p, d, dt, -1)
    ctx.tune(x, r, k, sketch=sk)
    tuned = {p: slso.tune_get(p, d, dt) for p in choices}
    print(f"[tune {kind} n={n} d={d} {sketch}] {tuned}", flush=True)
    takes_score = kind != "f32" and d % 16 == 0 and d <= 512 and k <= 64
    takes_cs = sketch == "countsketch"
    assert (0 <= tuned[slso.TUNE_SCORE] < 3) == takes_score
    assert (0 <= tuned[slso.TUNE_COUNTSKETCH] < 2) == takes_cs
    got, _ = ctx.leverage(x, 5, r, k, sketch=sk)
    assert np.array_equal(host(got).view(np.uint32), ref.view(np.uint32))
    for p in choices:
        slso.tune_set(p, d, dt, -1)
