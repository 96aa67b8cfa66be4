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
    assert lib.slso_create(None, 0) == slso.EINVAL
    h = ctypes.c_void_p()
    assert lib.slso_create(ctypes.byref(h), -1) == slso.EINVAL


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(slso, "_lib", None)
    with pytest.raises(ImportError):
        slso.load_library(str(tmp_path / "missing.so"))
