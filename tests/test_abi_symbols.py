"""The C-ABI library loads and exports every function include/sfcinpaint.h
declares (CPU only: no compute calls)."""
import ctypes
import os
import re
import struct

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
    assert lib.sfc_abi_version() == 2
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


class _Geometry(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("channels", ctypes.c_int32),
                ("shape", ctypes.c_int64 * 3)]


def _index_header(magic=b"SFCINDEX", nd=2, C=1, K=5, D=4, L=2, b=16, shape=(40, 44, 0), n=100,
                  S=5, mmax=10):
    # the header sfc_index_save writes: magic, version, 13 int32 (the last two
    # zero), 6 int64, 2 float, 2 uint64 (136 bytes, no padding)
    W64 = (D * b + 63) // 64
    ints = (nd, C, K, D, L, b, 0, 16, W64, S, mmax, 0, 0)
    return struct.pack("<8sI13i6q2f2Q", magic, 1, *ints, *shape, n, n, 1 << (b - 1),
                       0.0, 1.0, 0, 0)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_index_file_errors(tmp_path):
    """File and header errors of sfc_index_load are reported before any device
    work; so are sfc_index_save's argument errors."""
    lib = ctypes.CDLL(LIB)
    lib.sfc_last_error.restype = ctypes.c_char_p
    load = lib.sfc_index_load
    load.restype = ctypes.c_int
    load.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(_Geometry), ctypes.c_int32,
                     ctypes.c_void_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_void_p)]
    save = lib.sfc_index_save
    save.restype = ctypes.c_int
    save.argtypes = [ctypes.c_void_p, ctypes.c_char_p]
    assert len(_index_header()) == 136
    assert save(None, b"x") == -1
    g = _Geometry(2, 1, (ctypes.c_int64 * 3)(40, 44, 0))
    out = ctypes.c_void_p()
    p = ctypes.c_void_p(16)   # never dereferenced: every case fails before device work

    def run(data, K=5, geo=g):
        f = tmp_path / "i.sfc"
        f.write_bytes(data)
        rc = load(p, p, ctypes.byref(geo), K, None, str(f).encode(), ctypes.byref(out))
        assert rc == -1 and out.value is None
        return lib.sfc_last_error()

    assert load(p, p, ctypes.byref(g), 5, None, None, ctypes.byref(out)) == -1
    assert load(p, p, ctypes.byref(g), 5, None, str(tmp_path / "none").encode(),
                ctypes.byref(out)) == -1
    assert b"cannot open" in lib.sfc_last_error()
    assert b"not an index file" in run(b"")
    assert b"not an index file" in run(_index_header(magic=b"SFCINDEY"))
    assert b"another geometry" in run(_index_header(), K=7)
    assert b"another geometry" in run(_index_header(shape=(40, 45, 0)))
    assert b"another geometry" in run(_index_header(C=3))
    assert b"inconsistent" in run(_index_header(n=0))
    assert b"inconsistent" in run(_index_header(S=9))       # 2D has at most 8 subsets
    assert b"inconsistent" in run(_index_header(mmax=519))  # above the subset bound
    assert b"reduced_dim" in run(_index_header(D=30))
    assert b"truncated" in run(_index_header())
    # sums 25 * 8, bases 5 * 10 * 4, grid 5 * 4 * 8 + 5 * 8 bytes
    assert b"truncated" in run(_index_header() + b"\0" * 599)
    assert b"data after" in run(_index_header() + b"\0" * 601)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_options_layout_matches_the_header():
    # sfc_options_default is host-only; its struct_size is the C sizeof, and
    # the binding's mirror must have the same size and defaults
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None:
        pytest.skip("torch missing")
    from paper_1712_06326_amd import native
    o = native.Options()
    native.lib().sfc_options_default(ctypes.byref(o))
    assert o.struct_size == ctypes.sizeof(native.Options)
    assert (o.key_bits, o.window, o.curve, o.query_block, o.scan_variant, o.timing, o.norm) == \
        (8, 32, 0, 0, 0, 0, 0)
