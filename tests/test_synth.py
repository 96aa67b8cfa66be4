"""Input generators: the FP8 quantiser against torch's own float8_e4m3fn
conversion (an independent implementation), and its exact decode."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")


def test_fp8_codes_match_torch_float8():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((4000, 9)) * np.exp(2 * rng.standard_normal(9))
    x[:, 4] = 0.0
    codes, cs = synth.to_fp8_e4m3(x)
    assert cs[4] == 1.0
    v = x / cs.astype(np.float64)[None, :]
    ref = torch.from_numpy(v).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(codes, ref)


def test_fp8_decode_is_exact():
    codes = np.arange(256, dtype=np.uint8).reshape(1, 256)
    cs = np.ones(256, dtype=np.float32)
    got = synth.fp8_e4m3_to_f64(codes, cs)[0]
    ref = torch.from_numpy(codes[0].copy()).view(torch.float8_e4m3fn) \
        .to(torch.float64).numpy()
    finite = ~np.isnan(ref)
    assert np.array_equal(np.isnan(got), ~finite)
    assert np.array_equal(got[finite], ref[finite])
    # column max maps to the largest finite code, 448
    x = np.array([[1.0, -3.0], [0.5, 2.0]])
    c, s = synth.to_fp8_e4m3(x)
    assert c[0, 0] == 0x7E and c[1, 1] != 0 and c[0, 1] == 0xFE
