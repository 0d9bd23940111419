"""The C-ABI library loads and exports every function include/sfcinpaint.h
declares (CPU only: no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sfcinpaint.h")
LIB = os.path.join(ROOT, "paper_1712_06326_amd", "libsfcinpaint.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sfc_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("sfc_index_build", "sfc_query", "sfc_inpaint", "sfc_index_free",
                 "sfc_last_error", "sfc_fill_front", "sfc_extract_targets"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_only_calls():
    lib = ctypes.CDLL(LIB)
    lib.sfc_abi_version.restype = ctypes.c_int32
    assert lib.sfc_abi_version() == 1
    lib.sfc_last_error.restype = ctypes.c_char_p
    assert lib.sfc_last_error() == b""
    # argument errors are reported before any device work
    lib.sfc_index_build.restype = ctypes.c_int
    out = ctypes.c_void_p()
    rc = lib.sfc_index_build(None, None, None, 9, 8, 4, None, ctypes.byref(out))
    assert rc == -1 and b"geometry" in lib.sfc_last_error()
    lib.sfc_query.restype = ctypes.c_int
    assert lib.sfc_query(None, None, None, 1, 0, None, None) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_batch_argument_errors():
    lib = ctypes.CDLL(LIB)
    lib.sfc_batch_create.restype = ctypes.c_int
    lib.sfc_batch_query.restype = ctypes.c_int
    lib.sfc_last_error.restype = ctypes.c_char_p
    out = ctypes.c_void_p()
    arr = (ctypes.c_void_p * 1)(None)
    assert lib.sfc_batch_create(0, arr, arr, arr, 9, None, ctypes.byref(out)) == -1
    assert lib.sfc_batch_create(1, None, arr, arr, 9, None, ctypes.byref(out)) == -1
    geo = (ctypes.c_int32 * 8)(2, 1, 0, 0, 32, 0, 32, 0)
    assert lib.sfc_batch_create(1, arr, arr, geo, 4, None, ctypes.byref(out)) == -5
    assert b"K must be" in lib.sfc_last_error()
    assert lib.sfc_batch_query(None, None, None, None, None, None) == -1


def test_sort_pairs_argument_errors():
    lib = ctypes.CDLL(LIB)
    f = lib.sfc_sort_pairs
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                  ctypes.c_int32, ctypes.c_void_p]
    p = ctypes.c_void_p(16)   # never dereferenced: every case fails validation
    assert f(None, p, 10, 1, 1, None) == -1
    assert f(p, None, 10, 1, 1, None) == -1
    assert f(p, p, -1, 1, 1, None) == -1
    assert f(p, p, 10, 0, 1, None) == -1
    assert f(p, p, 10, 5, 1, None) == -1
    assert f(p, p, 10, 1, 0, None) == -1
    assert f(p, p, 1 << 32, 1, 1, None) == -5
    # n <= 1 is a no-op that touches nothing
    assert f(p, p, 1, 3, 2, None) == 0
    assert f(p, p, 0, 3, 2, None) == 0
