"""C-ABI checks that need no GPU: the library loads, exports every entry
point that ``include/slso.h`` declares, and rejects invalid arguments before
touching a device."""
import ctypes
import os
import re

import pytest

import paper_1812_07903_amd as slso

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "slso.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(slso_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(slso.LIB_PATH):
        from paper_1812_07903_amd import build
        build.build(verbose=False)
    return slso.load_library()


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("slso_sketch", "slso_leverage", "slso_order", "slso_create",
                 "slso_destroy"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(slso.EXPORTED) <= set(_declared())


def test_status_strings(lib):
    for st in (0, 1, -1, -2, -3, -4, -5):
        assert lib.slso_status_string(st)
    assert lib.slso_status_string(12345) == b"unknown status"


def test_invalid_arguments_rejected_without_device(lib):
    # NULL context / NULL outputs are rejected before any HIP call
    assert lib.slso_leverage(None, None, 1, 1, 1, None, None, None, None) == slso.EINVAL
    assert lib.slso_order(None, None, 5, None, None) == slso.EINVAL
    assert lib.slso_hash(1, 0, 0, 10, None, None, None) == slso.EINVAL
    assert lib.slso_hash(1, 16, -1, 10, None, None, None) == slso.EINVAL
    assert lib.slso_gaussian(1, 3, -1, 2, None, None) == slso.EINVAL
    assert lib.slso_create(None, 0, 0) == slso.EINVAL
    h = ctypes.c_void_p()
    assert lib.slso_create(ctypes.byref(h), -1, 0) == slso.EINVAL
    assert lib.slso_create(ctypes.byref(h), -1, 1 << 20) == slso.EINVAL


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(slso, "_lib", None)
    with pytest.raises(ImportError):
        slso.load_library(str(tmp_path / "missing.so"))


def _mat(n, d, dtype=slso.F32, fmt=slso.DENSE, col_scale=None):
    m = slso._Matrix()
    m.n, m.d, m.format, m.dtype = n, d, fmt, dtype
    m.values = 0x1000            # never dereferenced by the size query
    m.ld = d
    m.col_scale = col_scale
    return m


def _ws(lib, m, r, k, sketch=slso.COUNTSKETCH, refine=0, nnz=0, flags=0):
    opt = slso._Options(sketch, refine, 0.0, nnz, flags)
    out = ctypes.c_size_t()
    st = lib.slso_workspace_size(ctypes.byref(m), r, k, ctypes.byref(opt),
                                 ctypes.byref(out))
    return st, out.value


def test_workspace_size_is_a_host_computation(lib):
    n, d, r, k = 60000, 784, 16384, 64
    st, b = _ws(lib, _mat(n, d), r, k)
    assert st == slso.OK
    assert b % (2 << 20) == 0
    # at least the FP64 sketch, the partition arrays and R
    assert b >= r * d * 8 + 6 * n * 4 + d * d * 8
    st2, b2 = _ws(lib, _mat(n, d), r, k, refine=1)
    assert st2 == slso.OK and b2 >= b + 3 * d * d * 8 - (2 << 20)
    st3, b3 = _ws(lib, _mat(4000, 512, slso.BF16), 2048, 64,
                  sketch=slso.GAUSSIAN, refine=1)
    assert st3 == slso.OK and b3 >= 2048 * 512 * 4  # split-K partial sums


def test_workspace_size_osnap(lib):
    n, d, r, k = 60000, 784, 16384, 64
    _, b1 = _ws(lib, _mat(n, d), r, k)
    st, b2 = _ws(lib, _mat(n, d), r, k, sketch=slso.OSNAP)       # 2 per column
    assert st == slso.OK and b2 >= b1 + 6 * n * 4 - (2 << 20)
    st, b4 = _ws(lib, _mat(n, d), r, k, sketch=slso.OSNAP, nnz=4)
    assert st == slso.OK and b4 >= b2 + 12 * n * 4 - (2 << 20)
    assert _ws(lib, _mat(n, d), r, k, sketch=slso.OSNAP, nnz=1)[1] >= b1


def test_osnap_argument_errors(lib):
    m = _mat(100, 10)
    assert _ws(lib, m, 16, 4, sketch=slso.OSNAP, nnz=3)[0] == slso.EINVAL   # 3 does not divide 16
    assert _ws(lib, m, 32, 4, sketch=slso.OSNAP, nnz=32)[0] == slso.EINVAL  # above 16
    assert _ws(lib, m, 16, 4, sketch=slso.OSNAP, nnz=-1)[0] == slso.EINVAL
    assert _ws(lib, m, 16, 4, flags=8)[0] == slso.EINVAL                  # unknown flag
    assert _ws(lib, m, 16, 4, flags=slso.OPT_EPS_HAT)[0] == slso.OK
    assert _ws(lib, m, 16, 4, flags=slso.OPT_SVD_RANK)[0] == slso.OK
    assert _ws(lib, m, 16, 4, flags=slso.OPT_NO_SYNC)[0] == slso.OK


def test_no_sync_option_combinations(lib):
    """The device-decided path takes neither the refinement, the distortion
    report nor the SVD rank mode (each needs a host decision or read-back)."""
    m = _mat(1000, 16, slso.F32)
    ns = slso.OPT_NO_SYNC
    assert _ws(lib, m, 64, 4, flags=ns)[0] == slso.OK
    assert _ws(lib, m, 64, 4, sketch=slso.GAUSSIAN, flags=ns)[0] == slso.OK
    assert _ws(lib, m, 64, 4, refine=1, flags=ns)[0] == slso.EUNSUPPORTED
    assert _ws(lib, m, 64, 4, flags=ns | slso.OPT_EPS_HAT)[0] == slso.EUNSUPPORTED
    assert _ws(lib, m, 64, 4, flags=ns | slso.OPT_SVD_RANK)[0] == slso.EUNSUPPORTED
    assert _ws(lib, m, 16, 4, sketch=4)[0] == slso.EINVAL                # unknown sketch
    assert _ws(lib, m, 16, 4, sketch=slso.OSNAP, nnz=16)[0] == slso.OK


def test_srht_sizes_and_errors(lib):
    m = _mat(100, 10)                                     # n' = 128
    st, b = _ws(lib, m, 128, 4, sketch=slso.SRHT)
    assert st == slso.OK and b >= 128 * 10 * 8 + 128 * 10 * 8
    assert _ws(lib, m, 129, 4, sketch=slso.SRHT)[0] == slso.EINVAL      # r > n'
    c = _mat(100, 10, fmt=slso.CSR)
    c.row_ptr = ctypes.cast(0x3000, ctypes.c_void_p)     # never dereferenced
    c.col_idx = ctypes.cast(0x4000, ctypes.c_void_p)
    c.nnz = 10
    assert _ws(lib, c, 64, 4)[0] == slso.OK
    assert _ws(lib, c, 64, 4, sketch=slso.SRHT)[0] == slso.EUNSUPPORTED


def test_workspace_size_argument_errors(lib):
    assert _ws(lib, _mat(100, 10), 5, 4)[0] == slso.EINVAL          # r < d
    assert _ws(lib, _mat(100, 10), 16, -1)[0] == slso.EINVAL        # k < 0
    assert _ws(lib, _mat(0, 10), 16, 4)[0] == slso.EINVAL           # n < 1
    assert _ws(lib, _mat(100, 10, slso.F64), 16, 4,
               sketch=slso.GAUSSIAN)[0] == slso.EUNSUPPORTED
    assert _ws(lib, _mat(100, 10, slso.FP8_E4M3), 16, 4)[0] == slso.EUNSUPPORTED
    assert _ws(lib, _mat(100, 10, slso.F32, col_scale=0x2000), 16, 4)[0] == slso.EINVAL
    assert lib.slso_workspace_size(None, 16, 4, None, None) == slso.EINVAL


def test_server_rejects_invalid_arguments(lib):
    h = ctypes.c_void_p()
    assert lib.slso_server_create(None, 0, 2, 1 << 30) == slso.EINVAL
    assert lib.slso_server_create(ctypes.byref(h), 0, 0, 1 << 30) == slso.EINVAL
    assert lib.slso_server_create(ctypes.byref(h), 0, 65, 1 << 30) == slso.EINVAL
    assert lib.slso_server_create(ctypes.byref(h), 0, 2, 0) == slso.EINVAL
    assert lib.slso_server_submit(None, None, None) == slso.EINVAL
    assert lib.slso_server_poll(None, 1, None) == slso.EINVAL
    assert lib.slso_server_wait(None, 1, None) == slso.EINVAL
    assert lib.slso_server_stats(None, None) == slso.EINVAL
    assert lib.slso_server_destroy(None) == slso.EINVAL


# ---- binding checks: host tensors and wrong outputs never reach the kernels --
torch = pytest.importorskip("torch")


def test_binding_rejects_host_tensors():
    x = torch.zeros((10, 4), dtype=torch.float32)
    with pytest.raises(ValueError, match="GPU"):
        slso._matrix(x)
    with pytest.raises(ValueError, match="GPU"):
        slso._matrix(slso.Fp8Matrix(torch.zeros((10, 4), dtype=torch.uint8),
                                    torch.ones(4)))
    csr = slso.CsrMatrix(2, 3, torch.tensor([0, 1, 2]),
                         torch.tensor([0, 2], dtype=torch.int32),
                         torch.ones(2))
    with pytest.raises(ValueError, match="GPU"):
        slso._matrix(csr)
    with pytest.raises(TypeError):
        slso._matrix(x.numpy())


def test_binding_checks_outputs():
    # outputs are checked for device first, then dtype, size and layout
    with pytest.raises(ValueError, match="GPU"):
        slso._out(torch.empty(5, dtype=torch.float32), torch.float32, 5,
                  "cuda:0", "out")
    with pytest.raises(ValueError, match="GPU"):
        slso._out(torch.empty(5, dtype=torch.float64), torch.float32, 5,
                  "cuda:0", "out")
    with pytest.raises(ValueError, match="GPU"):
        slso._scores_in(torch.empty(5, dtype=torch.float32))
    with pytest.raises(ValueError):
        slso._f64_matrix(torch.empty((3, 3), dtype=torch.float64), "R")


def test_tune_table(lib):
    """The table of tuned launch shapes (host only): range checks, one entry
    per (pass, d, dtype), -1 removes."""
    ch = ctypes.c_int()
    assert lib.slso_tune_get(9, 64, 2, ctypes.byref(ch)) == slso.EINVAL
    assert lib.slso_tune_get(slso.TUNE_SCORE, 0, 2, ctypes.byref(ch)) == slso.EINVAL
    assert lib.slso_tune_get(slso.TUNE_SCORE, 64, 2, None) == slso.EINVAL
    assert lib.slso_tune_set(slso.TUNE_SCORE, 123, 2, 3) == slso.EINVAL
    assert lib.slso_tune_set(slso.TUNE_COUNTSKETCH, 123, 2, 2) == slso.EINVAL
    assert lib.slso_tune_set(slso.TUNE_SCORE, 123, 2, -2) == slso.EINVAL
    assert slso.tune_get(slso.TUNE_SCORE, 123, 2) == -1
    slso.tune_set(slso.TUNE_SCORE, 123, 2, 2)
    slso.tune_set(slso.TUNE_SCORE, 123, 3, 1)
    slso.tune_set(slso.TUNE_COUNTSKETCH, 123, 2, 0)
    assert slso.tune_get(slso.TUNE_SCORE, 123, 2) == 2
    assert slso.tune_get(slso.TUNE_SCORE, 123, 3) == 1
    assert slso.tune_get(slso.TUNE_COUNTSKETCH, 123, 2) == 0
    assert slso.tune_get(slso.TUNE_SCORE, 124, 2) == -1
    for p, dt in ((slso.TUNE_SCORE, 2), (slso.TUNE_SCORE, 3),
                  (slso.TUNE_COUNTSKETCH, 2)):
        slso.tune_set(p, 123, dt, -1)
        assert slso.tune_get(p, 123, dt) == -1
    assert lib.slso_tune(None, None, 16, 4, None, None) == slso.EINVAL
