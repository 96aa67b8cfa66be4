"""Python binding of libslso (sketched leverage scores on AMD MI355X).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libslso.so``; torch tensors supply device memory and streams.
The binding fails loudly when the library has not been built; there is no
CPU fallback.

Names mirror the C ABI (``include/slso.h``): ``sketch``, ``leverage``,
``order``, and the stage entry points ``hash``, ``gaussian``,
``gaussian_sketch_entries``, ``qr_r``, ``solve_upper`` and ``scores``.
Inputs: dense torch tensors (float64, float32, bfloat16), ``Fp8Matrix``
(e4m3fn codes with per-column scales) and ``CsrMatrix``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libslso.so")

# status codes (slso_status)
OK, RANK_DEFICIENT = 0, 1
EINVAL, ENOMEM, ENONFINITE, EDEVICE, EUNSUPPORTED = -1, -2, -3, -4, -5
# slso_dtype / slso_format / slso_sketch_kind
F64, F32, BF16, FP8_E4M3 = 0, 1, 2, 3
DENSE, CSR = 0, 1
COUNTSKETCH, GAUSSIAN, OSNAP, SRHT = 0, 1, 2, 3
OPT_SVD_RANK, OPT_EPS_HAT, OPT_NO_SYNC = 1, 2, 4
ORDER_DEC, ORDER_SWR, ORDER_SWOR = 0, 1, 2
TUNE_SCORE, TUNE_COUNTSKETCH = 0, 1
STREAM_GAUSS_S, STREAM_PI2 = 3, 4

EXPORTED = (
    "slso_create", "slso_destroy", "slso_status_string", "slso_last_error",
    "slso_sketch", "slso_sketch_svd", "slso_leverage", "slso_leverage_finish",
    "slso_order",
    "slso_order_sample",
    "slso_hash",
    "slso_gaussian", "slso_gaussian_sketch_entries",
    "slso_gaussian_sketch_entries_q", "slso_qr_r", "slso_qr_r_path",
    "slso_solve_upper", "slso_scores", "slso_scores_noalloc",
    "slso_workspace_size",
    "slso_tune", "slso_tune_get", "slso_tune_set",
    "slso_server_create", "slso_server_submit", "slso_server_poll",
    "slso_server_wait", "slso_server_stats", "slso_server_destroy",
    "slso_profile_enable", "slso_profile_read", "slso_profile_name",
    "slso_profile_only",
)
# slso_info.flags bits
INFO_REFINED, INFO_REFINE_FAILED = 1, 2
INFO_QR_SECOND_CHOLESKY, INFO_QR_HOUSEHOLDER, INFO_QR_TREE = 4, 8, 16
INFO_QR_ONE_PASS, INFO_RERUN = 32, 64
QR_AUTO, QR_PANEL, QR_TREE, QR_CHOLQR2, QR_CHOLQR2_FULL = 0, 1, 2, 3, 4


class SlsoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"slso status {status}: {msg}")
        self.status = status


class _Matrix(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("d", ctypes.c_int64),
        ("format", ctypes.c_int32), ("dtype", ctypes.c_int32),
        ("values", ctypes.c_void_p), ("ld", ctypes.c_int64),
        ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
        ("nnz", ctypes.c_int64),
        ("col_scale", ctypes.c_void_p), ("row_scale", ctypes.c_void_p),
    ]


class _Options(ctypes.Structure):
    _fields_ = [("sketch", ctypes.c_int32), ("refine", ctypes.c_int32),
                ("rank_tol", ctypes.c_double),
                ("nnz_per_col", ctypes.c_int32), ("flags", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int64), ("screen_full", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("diag_min", ctypes.c_double),
                ("diag_max", ctypes.c_double), ("eps_hat", ctypes.c_double)]


class _Job(ctypes.Structure):
    _fields_ = [("X", _Matrix), ("seed", ctypes.c_uint64), ("r", ctypes.c_int64),
                ("k", ctypes.c_int64), ("opt", _Options),
                ("scores", ctypes.c_void_p), ("perm", ctypes.c_void_p)]


class _JobResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("slot", ctypes.c_int32),
                ("info", _Info), ("submit_ms", ctypes.c_double),
                ("start_ms", ctypes.c_double), ("end_ms", ctypes.c_double)]


class _Counters(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_int64), ("running", ctypes.c_int64),
                ("max_running", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("allocated_bytes", ctypes.c_size_t),
                ("budget_bytes", ctypes.c_size_t)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libslso.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with paper_1812_07903_amd.build.build()")
    # torch first: it carries its own copy of the HIP runtime, and the library
    # must bind to that one (same soname) so that one runtime owns the device
    # and the library shares torch's memory and streams; loaded first, the
    # library would pull in the system runtime and torch a second one
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, i64, i32, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64
    sig = {
        "slso_create": ([ctypes.POINTER(vp), ctypes.c_int, ctypes.c_size_t],
                        ctypes.c_int),
        "slso_destroy": ([vp], ctypes.c_int),
        "slso_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "slso_last_error": ([vp], ctypes.c_char_p),
        "slso_sketch": ([vp, ctypes.POINTER(_Matrix), u64, i64,
                         ctypes.POINTER(_Options), vp, vp], ctypes.c_int),
        "slso_leverage": ([vp, ctypes.POINTER(_Matrix), u64, i64, i64,
                           ctypes.POINTER(_Options), vp, ctypes.POINTER(_Info),
                           vp], ctypes.c_int),
        "slso_leverage_finish": ([vp, ctypes.POINTER(_Info)], ctypes.c_int),
        "slso_order": ([vp, vp, i64, vp, vp], ctypes.c_int),
        "slso_order_sample": ([vp, vp, i64, i32, u64, ctypes.c_uint32, vp, vp],
                              ctypes.c_int),
        "slso_sketch_svd": ([vp, vp, u64, i64, vp, vp, vp, vp, vp], ctypes.c_int),
        "slso_hash": ([u64, i64, i64, i64, vp, vp, vp], ctypes.c_int),
        "slso_gaussian": ([u64, i32, i64, i64, vp, vp], ctypes.c_int),
        "slso_gaussian_sketch_entries": ([u64, i64, i64, i64, vp, vp],
                                         ctypes.c_int),
        "slso_gaussian_sketch_entries_q": ([u64, i32, i64, i64, i64, vp, vp],
                                           ctypes.c_int),
        "slso_qr_r": ([vp, vp, i64, i64, vp, vp], ctypes.c_int),
        "slso_qr_r_path": ([vp, vp, i64, i64, vp, ctypes.c_int, vp, vp],
                           ctypes.c_int),
        "slso_solve_upper": ([vp, vp, i64, vp, i64, vp], ctypes.c_int),
        "slso_scores": ([vp, ctypes.POINTER(_Matrix), vp, i64, vp, vp],
                        ctypes.c_int),
        "slso_scores_noalloc": ([vp, ctypes.POINTER(_Matrix), vp, i64, vp, vp],
                                ctypes.c_int),
        "slso_workspace_size": ([ctypes.POINTER(_Matrix), i64, i64,
                                 ctypes.POINTER(_Options),
                                 ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "slso_tune": ([vp, ctypes.POINTER(_Matrix), i64, i64,
                       ctypes.POINTER(_Options), vp], ctypes.c_int),
        "slso_tune_get": ([ctypes.c_int, i64, ctypes.c_int,
                           ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "slso_tune_set": ([ctypes.c_int, i64, ctypes.c_int, ctypes.c_int],
                          ctypes.c_int),
        "slso_server_create": ([ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int,
                                ctypes.c_size_t], ctypes.c_int),
        "slso_server_submit": ([vp, ctypes.POINTER(_Job),
                                ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
        "slso_server_poll": ([vp, i64, ctypes.POINTER(_JobResult)], ctypes.c_int),
        "slso_server_wait": ([vp, i64, ctypes.POINTER(_JobResult)], ctypes.c_int),
        "slso_server_stats": ([vp, ctypes.POINTER(_Counters)], ctypes.c_int),
        "slso_server_destroy": ([vp], ctypes.c_int),
        "slso_profile_enable": ([ctypes.c_int], ctypes.c_int),
        "slso_profile_read": ([vp, vp, ctypes.c_int], ctypes.c_int),
        "slso_profile_name": ([ctypes.c_int], ctypes.c_char_p),
        "slso_profile_only": ([ctypes.c_int], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


@dataclass
class CsrMatrix:
    """Device CSR matrix: row_ptr int64[n+1], col_idx int32[nnz], val f32."""
    n: int
    d: int
    row_ptr: object
    col_idx: object
    val: object


@dataclass
class Fp8Matrix:
    """Dense FP8-e4m3fn matrix: codes (n x d, uint8 or float8_e4m3fn, unit
    column stride) standing for e4m3(code) * col_scale[j] (float32[d])."""
    codes: object
    col_scale: object

    @property
    def shape(self):
        return self.codes.shape

    @property
    def device(self):
        return self.codes.device


def _rows(x) -> int:
    return x.n if isinstance(x, CsrMatrix) else x.shape[0]


def _cols(x) -> int:
    return x.d if isinstance(x, CsrMatrix) else x.shape[1]


def _device(x):
    return x.val.device if isinstance(x, CsrMatrix) else x.device


def _on_gpu(t, what: str):
    """Raise unless ``t`` is a torch tensor in device memory: the library
    reads and writes through device pointers only."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{what} must be on a GPU device, not {t.device}")


def _same_device(ts, what: str):
    devs = {t.device for t in ts if t is not None}
    if len(devs) > 1:
        raise ValueError(f"{what}: tensors on different devices {sorted(map(str, devs))}")


def _out(t, dtype, numel, device, what: str):
    """An output tensor: the given one after checks, or a new one of
    ``numel`` elements (an int, or a shape tuple)."""
    import math
    import torch
    shape = tuple(numel) if isinstance(numel, (tuple, list)) else (numel,)
    numel = math.prod(shape)
    if t is None:
        return torch.empty(shape, dtype=dtype, device=device)
    _on_gpu(t, what)
    if t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}, not {t.dtype}")
    if t.numel() != numel:
        raise ValueError(f"{what} must hold {numel} elements, not {t.numel()}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if torch.device(device) != t.device:
        raise ValueError(f"{what} is on {t.device}, the input on {device}")
    return t


def _matrix(x) -> _Matrix:
    import torch
    m = _Matrix()
    if isinstance(x, Fp8Matrix):
        _on_gpu(x.codes, "FP8 codes")
        _on_gpu(x.col_scale, "col_scale")
        _same_device((x.codes, x.col_scale), "FP8 matrix")
        c = x.codes
        if c.dtype not in (torch.uint8, torch.float8_e4m3fn):
            raise TypeError("FP8 codes must be uint8 or float8_e4m3fn")
        if c.dim() != 2 or c.stride(1) != 1:
            raise ValueError("FP8 codes must be 2-D with unit column stride")
        cs = x.col_scale
        if cs.dtype != torch.float32 or cs.numel() != c.shape[1] or \
                not cs.is_contiguous():
            raise TypeError("col_scale must be a contiguous float32[d]")
        m.n, m.d = c.shape
        m.format, m.dtype = DENSE, FP8_E4M3
        m.values = c.data_ptr()
        m.ld = c.stride(0)
        m.col_scale = cs.data_ptr()
        return m
    if isinstance(x, CsrMatrix):
        for t, w in ((x.row_ptr, "row_ptr"), (x.col_idx, "col_idx"),
                     (x.val, "CSR values")):
            _on_gpu(t, w)
            if not t.is_contiguous():
                raise ValueError(f"{w} must be contiguous")
        _same_device((x.row_ptr, x.col_idx, x.val), "CSR matrix")
        if x.row_ptr.numel() != x.n + 1 or x.col_idx.numel() != x.val.numel():
            raise ValueError("CSR needs n + 1 row pointers and one column "
                             "index per value")
        if x.val.dtype != torch.float32:
            raise TypeError("CSR values must be float32")
        if x.row_ptr.dtype != torch.int64 or x.col_idx.dtype != torch.int32:
            raise TypeError("CSR row_ptr must be int64 and col_idx int32")
        m.n, m.d, m.format, m.dtype = x.n, x.d, CSR, F32
        m.values = x.val.data_ptr()
        m.ld = x.d
        m.row_ptr = x.row_ptr.data_ptr()
        m.col_idx = x.col_idx.data_ptr()
        m.nnz = int(x.col_idx.numel())
        return m
    _on_gpu(x, "X")
    if x.dim() != 2 or x.stride(1) != 1:
        raise ValueError("dense X must be 2-D with unit column stride")
    code = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}.get(x.dtype)
    if code is None:
        raise TypeError(f"unsupported dtype {x.dtype}")
    m.n, m.d = x.shape
    m.format, m.dtype = DENSE, code
    m.values = x.data_ptr()
    m.ld = x.stride(0)
    return m


def _check(st: int, ctx=None):
    if st < 0:
        lib = load_library()
        msg = lib.slso_last_error(ctx).decode() if ctx else ""
        if not msg:
            msg = lib.slso_status_string(st).decode()
        raise SlsoError(st, msg)
    return st


class Context:
    """Owns a library context (device workspace) on one HIP device.
    ``workspace_bytes`` > 0 allocates that workspace once (calls that need
    more fail with ENOMEM); 0 lets it grow on demand."""

    def __init__(self, device: int = 0, workspace_bytes: int = 0):
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.slso_create(ctypes.byref(h), device, workspace_bytes))
        self._h = h
        self.device = device

    @property
    def handle(self):
        return self._h

    def _here(self, dev):
        """Raise unless ``dev`` is this context's device."""
        idx = dev.index if dev.index is not None else 0
        if dev.type != "cuda" or idx != self.device:
            raise ValueError(f"tensor on {dev}, context on cuda:{self.device}")

    def close(self):
        if self._h:
            load_library().slso_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- hot path ----------------------------------------------------------
    def sketch(self, x, seed: int, r: int, sketch: int = COUNTSKETCH, out=None,
               stream=None, nnz: int = 0):
        import torch
        m = _matrix(x)
        self._here(_device(x))
        out = _out(out, torch.float64, (r, _cols(x)), _device(x), "out")
        opt = _Options(sketch, 0, 0.0, nnz, 0)
        _check(load_library().slso_sketch(self._h, ctypes.byref(m), seed, r,
                                          ctypes.byref(opt), _ptr(out),
                                          _stream(stream)), self._h)
        return out

    def leverage(self, x, seed: int, r: int, k: int, sketch: int = COUNTSKETCH,
                 refine: bool = False, rank_tol: float = 0.0, out=None,
                 stream=None, nnz: int = 0, svd_rank: bool = False,
                 eps_hat: bool = False, no_sync: bool = False):
        """Scores (float32 device tensor) and the rank-decision info dict.
        ``nnz``: OSNAP nonzeros per column of S (0 selects 2); ``svd_rank``:
        decide the rank by the SVD of R every time; ``eps_hat``: report the
        sketch's realised distortion on range(X) as info["eps_hat"];
        ``no_sync``: enqueue the whole job (capturable) and return (out,
        None); leverage_finish() then gives the info dict."""
        import torch
        m = _matrix(x)
        self._here(_device(x))
        out = _out(out, torch.float32, _rows(x), _device(x), "out")
        opt = _Options(sketch, 1 if refine else 0, rank_tol, nnz,
                       (OPT_SVD_RANK if svd_rank else 0) |
                       (OPT_EPS_HAT if eps_hat else 0) |
                       (OPT_NO_SYNC if no_sync else 0))
        info = _Info()
        st = _check(load_library().slso_leverage(
            self._h, ctypes.byref(m), seed, r, k, ctypes.byref(opt), _ptr(out),
            ctypes.byref(info), _stream(stream)), self._h)
        if no_sync:
            self._keep = (x, m, out)  # the pending call's buffers
            return out, None
        return out, _info_dict(info, st)

    def tune(self, x, r: int, k: int, sketch: int = COUNTSKETCH, nnz: int = 0,
             stream=None):
        """Time the tunable launch shapes of slso_leverage on x and record
        the fastest per (pass, d, dtype) (slso_tune; results do not depend
        on the choice)."""
        m = _matrix(x)
        self._here(_device(x))
        opt = _Options(sketch, 0, 0.0, nnz, 0)
        _check(load_library().slso_tune(self._h, ctypes.byref(m), r, k,
                                        ctypes.byref(opt), _stream(stream)),
               self._h)

    def leverage_finish(self):
        """Info dict of the pending no-sync leverage call (waits for its
        stream; a case the device path does not take is rerun there)."""
        info = _Info()
        st = _check(load_library().slso_leverage_finish(self._h,
                                                        ctypes.byref(info)),
                    self._h)
        self._keep = None
        return _info_dict(info, st)

    def order(self, scores, out=None, stream=None):
        import torch
        _scores_in(scores)
        self._here(scores.device)
        out = _out(out, torch.int32, scores.numel(), scores.device, "out")
        _check(load_library().slso_order(self._h, _ptr(scores), scores.numel(),
                                         _ptr(out), _stream(stream)), self._h)
        return out

    def sketch_svd(self, x, seed: int, r: int, sketch: int = COUNTSKETCH,
                   nnz: int = 0, stream=None):
        """Sketched SVD of S X: (sigma descending, V with column j the right
        singular vector of sigma[j]) as float64 device tensors."""
        import torch
        d = _cols(x)
        m = _matrix(x)
        self._here(_device(x))
        sx = torch.empty((r, d), dtype=torch.float64, device=_device(x))
        sigma = torch.empty(d, dtype=torch.float64, device=_device(x))
        v = torch.empty((d, d), dtype=torch.float64, device=_device(x))
        opt = _Options(sketch, 0, 0.0, nnz, 0)
        _check(load_library().slso_sketch_svd(
            self._h, ctypes.byref(m), seed, r, ctypes.byref(opt), _ptr(sx),
            _ptr(sigma), _ptr(v), _stream(stream)), self._h)
        return sigma, v

    def order_sample(self, scores, policy: int, seed: int, epoch: int = 0,
                     out=None, stream=None):
        """One epoch's order by a sampling policy (ORDER_DEC, ORDER_SWR with
        replacement, ORDER_SWOR without): int32 row indices."""
        import torch
        _scores_in(scores)
        self._here(scores.device)
        out = _out(out, torch.int32, scores.numel(), scores.device, "out")
        _check(load_library().slso_order_sample(
            self._h, _ptr(scores), scores.numel(), policy, seed, epoch,
            _ptr(out), _stream(stream)), self._h)
        return out

    # ---- stages ---------------------------------------------------------------
    def qr_r(self, a, stream=None):
        """R (non-negative diagonal) of a QR of ``a``, which is overwritten."""
        return self.qr_r_path(a, QR_AUTO, stream)[0]

    def qr_r_path(self, a, path=QR_AUTO, stream=None):
        """(R, path used) starting from ``path`` (QR_AUTO, QR_PANEL or
        QR_TREE); ``a`` is overwritten."""
        import torch
        _f64_matrix(a, "a")
        self._here(a.device)
        m, d = a.shape
        r = torch.empty((d, d), dtype=torch.float64, device=a.device)
        used = ctypes.c_int32(-1)
        _check(load_library().slso_qr_r_path(self._h, _ptr(a), m, d, _ptr(r),
                                             int(path), ctypes.byref(used),
                                             _stream(stream)), self._h)
        return r, used.value

    def solve_upper(self, r, b, stream=None):
        """Solve R X = B in place (B is d x k, float64)."""
        _f64_matrix(r, "R")
        _f64_matrix(b, "B")
        self._here(r.device)
        self._here(b.device)
        if r.shape[0] != r.shape[1] or r.shape[0] != b.shape[0]:
            raise ValueError("R must be d x d and B d x k")
        d, k = b.shape
        _check(load_library().slso_solve_upper(self._h, _ptr(r), d, _ptr(b), k,
                                               _stream(stream)), self._h)
        return b

    def scores(self, x, m, out=None, stream=None, noalloc=False):
        """l_i = ||x_i M||^2 (slso_scores). noalloc=True calls
        slso_scores_noalloc: no device allocation, the library's fixed
        per-device scratch instead of the context workspace (calls that
        overlap on one GPU race on it)."""
        import torch
        mm = _matrix(x)
        self._here(_device(x))
        _on_gpu(m, "M")
        if m.dtype != torch.float64 or m.dim() != 2 or not m.is_contiguous() \
                or m.shape[0] != _cols(x):
            raise ValueError("M must be a contiguous float64 d x k tensor")
        self._here(m.device)
        out = _out(out, torch.float32, _rows(x), _device(x), "out")
        lib = load_library()
        fn = lib.slso_scores_noalloc if noalloc else lib.slso_scores
        _check(fn(self._h, ctypes.byref(mm), _ptr(m), m.shape[1], _ptr(out),
                  _stream(stream)), self._h)
        return out


def _f64_matrix(a, what: str):
    import torch
    _on_gpu(a, what)
    if a.dtype != torch.float64 or a.dim() != 2 or not a.is_contiguous():
        raise ValueError(f"{what} must be a contiguous 2-D float64 tensor")


def _scores_in(scores):
    import torch
    _on_gpu(scores, "scores")
    if scores.dtype != torch.float32 or not scores.is_contiguous():
        raise TypeError("scores must be a contiguous float32 tensor")


def _info_dict(info, st):
    return {"status": st, "rank": info.rank,
            "screen_full": bool(info.screen_full), "flags": info.flags,
            "refined": bool(info.flags & INFO_REFINED),
            "diag_min": info.diag_min, "diag_max": info.diag_max,
            "eps_hat": info.eps_hat}


def tune_get(pass_: int, d: int, dtype: int) -> int:
    """The recorded launch-shape choice for (pass, d, slso dtype), or -1."""
    ch = ctypes.c_int()
    _check(load_library().slso_tune_get(pass_, d, dtype, ctypes.byref(ch)))
    return ch.value


def tune_set(pass_: int, d: int, dtype: int, choice: int) -> None:
    """Record a launch-shape choice by hand (-1 removes it)."""
    _check(load_library().slso_tune_set(pass_, d, dtype, choice))


def workspace_size(x, r: int, k: int, sketch: int = COUNTSKETCH,
                   refine: bool = False, rank_tol: float = 0.0,
                   nnz: int = 0) -> int:
    """Device workspace bytes a context allocates for leverage + order."""
    m = _matrix(x)
    opt = _Options(sketch, 1 if refine else 0, rank_tol, nnz, 0)
    out = ctypes.c_size_t()
    _check(load_library().slso_workspace_size(ctypes.byref(m), r, k,
                                              ctypes.byref(opt),
                                              ctypes.byref(out)))
    return out.value


class Ticket:
    """A submitted job: keeps its input and outputs alive until collected."""

    def __init__(self, tid, x, scores, perm):
        self.id = tid
        self.x = x
        self.scores = scores
        self.perm = perm


class Server:
    """Serving loop of the C ABI (slso_server_*): ``slots`` concurrent jobs
    admitted under an HBM budget for the slots' workspaces."""

    def __init__(self, device: int = 0, slots: int = 4,
                 hbm_budget: int = 64 << 30):
        h = ctypes.c_void_p()
        _check(load_library().slso_server_create(ctypes.byref(h), device, slots,
                                                 hbm_budget))
        self._h = h

    def submit(self, x, seed: int, r: int, k: int, sketch: int = COUNTSKETCH,
               refine: bool = False, rank_tol: float = 0.0, order: bool = True,
               scores=None, perm=None, nnz: int = 0) -> Ticket:
        """Queue a job; X must already hold its values (synchronise first)."""
        import torch
        n = _rows(x)
        jx = _matrix(x)
        scores = _out(scores, torch.float32, n, _device(x), "scores")
        if order:
            perm = _out(perm, torch.int32, n, _device(x), "perm")
        job = _Job()
        job.X = jx
        job.seed, job.r, job.k = seed, r, k
        job.opt = _Options(sketch, 1 if refine else 0, rank_tol, nnz, 0)
        job.scores = scores.data_ptr()
        job.perm = perm.data_ptr() if order else None
        tid = ctypes.c_int64()
        _check(load_library().slso_server_submit(self._h, ctypes.byref(job),
                                                 ctypes.byref(tid)))
        return Ticket(tid.value, x, scores, perm if order else None)

    @staticmethod
    def _result(res):
        return {"status": res.status, "slot": res.slot,
                "info": _info_dict(res.info, res.status),
                "submit_ms": res.submit_ms, "start_ms": res.start_ms,
                "end_ms": res.end_ms,
                "latency_ms": res.end_ms - res.submit_ms}

    def poll(self, t: Ticket):
        """None while running, else the result dict (ticket retired)."""
        res = _JobResult()
        st = _check(load_library().slso_server_poll(self._h, t.id,
                                                    ctypes.byref(res)))
        return self._result(res) if st == 1 else None

    def wait(self, t: Ticket) -> dict:
        res = _JobResult()
        _check(load_library().slso_server_wait(self._h, t.id, ctypes.byref(res)))
        return self._result(res)

    def stats(self) -> dict:
        c = _Counters()
        _check(load_library().slso_server_stats(self._h, ctypes.byref(c)))
        return {f: getattr(c, f) for f, _ in _Counters._fields_}

    def close(self):
        if self._h:
            load_library().slso_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def profile_enable(on: bool = True) -> None:
    """Record HIP events around every library kernel launch (process-wide)."""
    load_library().slso_profile_enable(1 if on else 0)


def profile_only(name=None) -> None:
    """Record only the kernel called ``name`` (None: every kernel)."""
    lib = load_library()
    kid = -1
    if name is not None:
        names = [lib.slso_profile_name(i).decode() for i in range(64)]
        if name not in names:
            raise ValueError(f"unknown kernel {name!r}")
        kid = names.index(name)
    _check(lib.slso_profile_only(kid))


def profile_read() -> dict:
    """{kernel name: (total ms, launches)} since the last read; synchronises."""
    lib = load_library()
    n = 64
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    k = lib.slso_profile_read(ms, cnt, n)
    if k < 0:
        raise SlsoError(k, "profile read failed")
    return {lib.slso_profile_name(i).decode(): (ms[i], cnt[i]) for i in range(k)}


def hash(seed: int, r: int, n: int, row0: int = 0, device="cuda", stream=None):
    """CountSketch bucket (int32) and sign (int8) of rows row0..row0+n-1."""
    import torch
    b = torch.empty(n, dtype=torch.int32, device=device)
    s = torch.empty(n, dtype=torch.int8, device=device)
    _check(load_library().slso_hash(seed, r, row0, n, _ptr(b), _ptr(s),
                                    _stream(stream)))
    return b, s


def gaussian(seed: int, stream_id: int, rows: int, cols: int, device="cuda",
             stream=None):
    """Gaussian stream entries z(a, b), a < rows, b < cols (float64)."""
    import torch
    out = torch.empty((rows, cols), dtype=torch.float64, device=device)
    _check(load_library().slso_gaussian(seed, stream_id, rows, cols, _ptr(out),
                                        _stream(stream)))
    return out


def gaussian_sketch_entries(seed: int, r: int, n: int, row0: int = 0,
                            device="cuda", stream=None):
    """FP32 Gaussian sketch entries G[j][row0 + i] (r x n float32)."""
    import torch
    out = torch.empty((r, n), dtype=torch.float32, device=device)
    _check(load_library().slso_gaussian_sketch_entries(seed, r, row0, n,
                                                       _ptr(out),
                                                       _stream(stream)))
    return out


def gaussian_sketch_entries_q(seed: int, dtype: int, r: int, n: int,
                              row0: int = 0, device="cuda", stream=None):
    """Quantile-form Gaussian sketch entries G[j][row0 + i] of the BF16
    (``dtype=BF16``) or FP8 (``dtype=FP8_E4M3``) input path, as an r x n
    float32 tensor."""
    import torch
    out = torch.empty((r, n), dtype=torch.float32, device=device)
    _check(load_library().slso_gaussian_sketch_entries_q(
        seed, dtype, r, row0, n, _ptr(out), _stream(stream)))
    return out
