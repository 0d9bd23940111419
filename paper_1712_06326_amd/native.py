"""Thin Python binding of libsfcinpaint.so (argument marshalling only).

Every computation happens in the HIP library; this module only turns torch
tensors into device pointers and sizes and checks status codes. PyTorch is
used for device memory and streams. If the library is missing this module
raises at import time: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsfcinpaint.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
        "or `python paper_1712_06326_amd/build.py` first")

_L = C.CDLL(LIB_PATH)

SFC_OK, SFC_EINVAL, SFC_ENOMEM, SFC_EDEVICE, SFC_EEMPTY, SFC_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
MODES = {"fp32": 0, "bf16": 1, "fp8": 2, "index": 3}
CURVES = {"morton": 0, "hilbert": 1}
ORDERS = {"criminisi": 0, "raster": 1}


class Geometry(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("channels", C.c_int32), ("shape", C.c_int64 * 3)]


class Options(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("key_bits", C.c_int32), ("window", C.c_int32),
                ("curve", C.c_int32),
                ("query_block", C.c_int32), ("scan_variant", C.c_int32), ("stream", C.c_void_p),
                ("timing", C.c_int32), ("norm", C.c_int32)]


class WindowTrial(C.Structure):
    _fields_ = [("window", C.c_int32), ("recall", C.c_float), ("accel_error", C.c_float),
                ("ms", C.c_float)]


class KernelTime(C.Structure):
    _fields_ = [("kernel", C.c_char_p), ("launches", C.c_int32), ("ms", C.c_float)]


class IndexInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_sub", C.c_int64), ("ndim", C.c_int32),
                ("channels", C.c_int32), ("K", C.c_int32), ("P", C.c_int32),
                ("has_sfc", C.c_int32), ("n_subsets", C.c_int32), ("reduced_dim", C.c_int32),
                ("n_curves", C.c_int32), ("key_bits", C.c_int32), ("key_words", C.c_int32),
                ("window", C.c_int32), ("curve", C.c_int32), ("vmin", C.c_float),
                ("qscale", C.c_float)]


class FillLog(C.Structure):
    _fields_ = [("cap", C.c_int64), ("len", C.c_int64), ("centre_host", C.c_void_p),
                ("source_host", C.c_void_p), ("cost_host", C.c_void_p)]


P = C.c_void_p
I32, I64 = C.c_int32, C.c_int64
ST = C.c_int
_SIG = {
    "sfc_abi_version": (I32, []),
    "sfc_last_error": (C.c_char_p, []),
    "sfc_options_default": (None, [C.POINTER(Options)]),
    "sfc_fill_front": (ST, [P, C.POINTER(Geometry), P, I64, C.POINTER(C.c_int64), P]),
    "sfc_extract_targets": (ST, [P, P, C.POINTER(Geometry), I32, P, I64, P, P, P]),
    "sfc_dictionary_build": (ST, [P, P, C.POINTER(Geometry), I32, C.POINTER(Options),
                                  C.POINTER(P)]),
    "sfc_index_build": (ST, [P, P, C.POINTER(Geometry), I32, I32, I32, C.POINTER(Options),
                             C.POINTER(P)]),
    "sfc_index_build_with_basis": (ST, [P, P, C.POINTER(Geometry), I32, I32, I32,
                                        C.POINTER(Options), P, C.POINTER(P)]),
    "sfc_query": (ST, [P, P, P, I64, C.c_int, P, P]),
    "sfc_query_fp32_noalloc": (ST, [P, P, P, I64, P, P]),
    "sfc_noalloc_bytes": (I64, [P, I64]),
    "sfc_query_candidates": (ST, [P, P, P, I64, P, P]),
    "sfc_query_knn": (ST, [P, P, P, I64, I32, I32, P, P, P, P]),
    "sfc_query_coords": (ST, [P, P, P, I64, P, P]),
    "sfc_query_stats": (ST, [P, C.POINTER(C.c_int64)]),
    "sfc_query_kernel_times": (ST, [P, P, I32, C.POINTER(C.c_int32)]),
    "sfc_set_timing": (ST, [P, I32]),
    "sfc_query_filter_tiles": (ST, [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "sfc_autotune_window": (ST, [P, P, P, I64, C.c_float, C.c_float, P, I32,
                                 C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "sfc_autotune": (ST, [P, P, P, I64, C.POINTER(C.c_int32)]),
    "sfc_index_info_get": (ST, [P, C.POINTER(IndexInfo)]),
    "sfc_index_dictionary": (ST, [P, P]),
    "sfc_index_quantized": (ST, [P, P]),
    "sfc_index_get_basis": (ST, [P, I32, P, C.POINTER(C.c_int32)]),
    "sfc_index_get_params": (ST, [P, I32, P, C.POINTER(C.c_int64)]),
    "sfc_index_projection": (ST, [P, I32, P]),
    "sfc_index_export": (ST, [P, I32, I32, P, P]),
    "sfc_index_free": (None, [P]),
    "sfc_index_save": (ST, [P, C.c_char_p]),
    "sfc_index_load": (ST, [P, P, C.POINTER(Geometry), I32, C.POINTER(Options), C.c_char_p,
                            C.POINTER(P)]),
    "sfc_sort_pairs": (ST, [P, P, I64, I32, I32, P]),
    "sfc_debug_fail_alloc": (None, [I64]),
    "sfc_debug_list_capacity": (None, [I32]),
    "sfc_batch_create": (ST, [I32, P, P, P, I32, C.POINTER(Options), C.POINTER(P)]),
    "sfc_batch_query": (ST, [P, P, P, P, P, P]),
    "sfc_batch_autotune": (ST, [P, P, P, P, P, P, C.POINTER(C.c_int32)]),
    "sfc_batch_stats": (ST, [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                             C.POINTER(C.c_int32)]),
    "sfc_batch_free": (None, [P]),
    "sfc_inpaint": (ST, [P, P, C.POINTER(Geometry), I32, C.c_int, C.c_int, P,
                         C.POINTER(Options), C.POINTER(C.c_int64), C.POINTER(FillLog)]),
}
for _name, (_res, _args) in _SIG.items():
    _f = getattr(_L, _name)
    _f.restype = _res
    _f.argtypes = _args


class SfcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sfc status {code}: {msg}")
        self.code = code


def _check(code):
    if code != SFC_OK:
        raise SfcError(code, _L.sfc_last_error().decode())


def lib():
    return _L


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def geometry(mask: torch.Tensor, channels: int) -> Geometry:
    g = Geometry()
    g.ndim = mask.dim()
    g.channels = channels
    for i, s in enumerate(mask.shape):
        g.shape[i] = s
    return g


NORMS = {"l2": 0, "l1": 1}


def options(key_bits=8, window=32, curve="morton", query_block=0, scan_variant=0,
            timing=False, norm="l2") -> Options:
    o = Options()
    _L.sfc_options_default(C.byref(o))
    o.key_bits = key_bits
    o.window = window
    o.curve = CURVES[curve] if isinstance(curve, str) else int(curve)
    o.query_block = query_block
    o.scan_variant = scan_variant
    o.stream = _stream()
    o.timing = 1 if timing else 0
    o.norm = NORMS[norm] if isinstance(norm, str) else int(norm)
    return o


def debug_fail_alloc(n: int) -> None:
    """Makes the library's n-th device allocation from now fail (0: off)."""
    _L.sfc_debug_fail_alloc(n)


def debug_list_capacity(cap: int) -> None:
    """Forces the reduced-precision scan's per-query list capacity (0: automatic)."""
    _L.sfc_debug_list_capacity(cap)


def fill_front(mask: torch.Tensor) -> torch.Tensor:
    g = geometry(mask, 1)
    n = C.c_int64()
    _check(_L.sfc_fill_front(_ptr(mask), C.byref(g), None, 0, C.byref(n), _stream()))
    out = torch.empty(max(n.value, 1), dtype=torch.int64, device=mask.device)
    _check(_L.sfc_fill_front(_ptr(mask), C.byref(g), _ptr(out), n.value, C.byref(n), _stream()))
    return out[:n.value]


def sort_pairs(keys: torch.Tensor, ids: torch.Tensor) -> None:
    """Sorts in place, per array, (key, id) pairs by key (stable): keys int64
    [arrays, key_words, n] holding the uint64 words (word 0 most
    significant), ids int32 [arrays, n]."""
    if keys.dim() != 3 or ids.dim() != 2 or keys.dtype != torch.int64 or ids.dtype != torch.int32:
        raise ValueError("keys int64 [arrays, key_words, n], ids int32 [arrays, n]")
    arrays, words, n = keys.shape
    if tuple(ids.shape) != (arrays, n) or not keys.is_contiguous() or not ids.is_contiguous():
        raise ValueError("ids must be [arrays, n]; both contiguous")
    _check(_L.sfc_sort_pairs(_ptr(keys), _ptr(ids), n, words, arrays, _stream()))


def extract_targets(volume: torch.Tensor, mask: torch.Tensor, K: int, centres: torch.Tensor):
    Cc = volume.shape[-1]
    Q = centres.numel()
    Kd = K ** mask.dim()
    t = torch.empty((Q, Kd, Cc), dtype=torch.float32, device=volume.device)
    m = torch.empty((Q, Kd), dtype=torch.uint8, device=volume.device)
    g = geometry(mask, Cc)
    _check(_L.sfc_extract_targets(_ptr(volume), _ptr(mask), C.byref(g), K, _ptr(centres), Q,
                                  _ptr(t), _ptr(m), _stream()))
    return t, m


class Index:
    """Owner of an sfc_index handle. The volume tensor is kept referenced for
    the handle's lifetime (the library reads dictionary patches in place)."""

    def __init__(self, volume: torch.Tensor, mask: torch.Tensor, K: int, reduced_dim: int = 0,
                 n_curves: int = 0, bases: list | None = None, **opts):
        self.volume, self.mask, self.K = volume, mask, K
        self._opts = options(**opts)
        g = geometry(mask, volume.shape[-1])
        h = C.c_void_p()
        if reduced_dim <= 0:
            _check(_L.sfc_dictionary_build(_ptr(volume), _ptr(mask), C.byref(g), K,
                                           C.byref(self._opts), C.byref(h)))
        elif bases is None:
            _check(_L.sfc_index_build(_ptr(volume), _ptr(mask), C.byref(g), K, reduced_dim,
                                      n_curves, C.byref(self._opts), C.byref(h)))
        else:
            import numpy as np
            flat = np.ascontiguousarray(np.concatenate([np.asarray(b, np.int8).ravel()
                                                        for b in bases]))
            _check(_L.sfc_index_build_with_basis(
                _ptr(volume), _ptr(mask), C.byref(g), K, reduced_dim, n_curves,
                C.byref(self._opts), flat.ctypes.data_as(C.c_void_p), C.byref(h)))
        self._h = h

    @classmethod
    def load(cls, volume: torch.Tensor, mask: torch.Tensor, K: int, path: str, **opts):
        """A handle from a file written by save() for the same volume and mask."""
        self = cls.__new__(cls)
        self.volume, self.mask, self.K = volume, mask, K
        self._opts = options(**opts)
        g = geometry(mask, volume.shape[-1])
        h = C.c_void_p()
        _check(_L.sfc_index_load(_ptr(volume), _ptr(mask), C.byref(g), K, C.byref(self._opts),
                                 str(path).encode(), C.byref(h)))
        self._h = h
        return self

    def save(self, path: str) -> None:
        _check(_L.sfc_index_save(self._h, str(path).encode()))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _L.sfc_index_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def info(self) -> IndexInfo:
        i = IndexInfo()
        _check(_L.sfc_index_info_get(self._h, C.byref(i)))
        return i

    def dictionary(self) -> torch.Tensor:
        out = torch.empty(self.info.n, dtype=torch.int64, device=self.volume.device)
        _check(_L.sfc_index_dictionary(self._h, _ptr(out)))
        return out

    def query(self, t: torch.Tensor, m: torch.Tensor, mode: str = "fp32"):
        Q = m.shape[0]
        bi = torch.empty(Q, dtype=torch.int64, device=t.device)
        bc = torch.empty(Q, dtype=torch.float32, device=t.device)
        _check(_L.sfc_query(self._h, _ptr(t), _ptr(m), Q, MODES[mode], _ptr(bi), _ptr(bc)))
        return bi, bc

    def query_noalloc(self, t: torch.Tensor, m: torch.Tensor, best_id: torch.Tensor,
                      best_cost: torch.Tensor) -> None:
        """The float32 full scan into caller-allocated outputs, through the
        entry point that allocates nothing (sfc_query_fp32_noalloc)."""
        _check(_L.sfc_query_fp32_noalloc(self._h, _ptr(t), _ptr(m), m.shape[0], _ptr(best_id),
                                         _ptr(best_cost)))

    def noalloc_bytes(self, Q: int) -> int:
        return int(_L.sfc_noalloc_bytes(self._h, Q))

    def knn(self, t: torch.Tensor, m: torch.Tensor, k: int = 80, mu: int = 256,
            candidates: bool = False):
        """Exact k-NN query (Section II.D): (best_id, best_cost), plus
        (cand [Q, k] ascending ids padded -1, ncand [Q]) if candidates."""
        Q = m.shape[0]
        bi = torch.empty(Q, dtype=torch.int64, device=t.device)
        bc = torch.empty(Q, dtype=torch.float32, device=t.device)
        cand = torch.empty((Q, k), dtype=torch.int64, device=t.device) if candidates else None
        nc = torch.empty(Q, dtype=torch.int32, device=t.device) if candidates else None
        _check(_L.sfc_query_knn(self._h, _ptr(t), _ptr(m), Q, k, mu, _ptr(bi), _ptr(bc),
                                _ptr(cand), _ptr(nc)))
        return (bi, bc, cand, nc) if candidates else (bi, bc)

    def autotune(self, t: torch.Tensor, m: torch.Tensor) -> int:
        """Picks the fastest float32-scan tile shape on these targets."""
        v = C.c_int32()
        _check(_L.sfc_autotune(self._h, _ptr(t), _ptr(m), m.shape[0], C.byref(v)))
        return v.value

    def autotune_window(self, t: torch.Tensor, m: torch.Tensor, target_recall: float = 0.9,
                        max_accel_error: float = -1.0):
        """Smallest window reaching target_recall (and an acceleration error
        of at most max_accel_error, if >= 0) against the float32 scan on
        these targets; set on the handle. Returns (window, [trials])."""
        cap = 32
        arr = (WindowTrial * cap)()
        n, w = C.c_int32(), C.c_int32()
        _check(_L.sfc_autotune_window(self._h, _ptr(t), _ptr(m), m.shape[0],
                                      C.c_float(target_recall), C.c_float(max_accel_error),
                                      C.cast(arr, C.c_void_p), cap, C.byref(n), C.byref(w)))
        trials = [{"window": arr[i].window, "recall": arr[i].recall,
                   "accel_error": arr[i].accel_error, "ms": arr[i].ms}
                  for i in range(min(n.value, cap))]
        return w.value, trials

    def set_timing(self, on: bool) -> None:
        """Records kernel durations of the next queries (or stops)."""
        _check(_L.sfc_set_timing(self._h, 1 if on else 0))

    def kernel_times(self) -> dict:
        """{kernel: (launches, total ms)} of the timed queries since the last
        read (timing=True); reading clears them."""
        cap = 16
        arr = (KernelTime * cap)()
        n = C.c_int32()
        _check(_L.sfc_query_kernel_times(self._h, arr, cap, C.byref(n)))
        return {arr[i].kernel.decode(): (arr[i].launches, arr[i].ms)
                for i in range(min(n.value, cap))}

    def filter_tiles(self):
        """(pass-1 tiles, pass-2 tiles) of the last bf16 query."""
        a, b = C.c_int64(), C.c_int64()
        _check(_L.sfc_query_filter_tiles(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def fallbacks(self) -> int:
        n = C.c_int64()
        _check(_L.sfc_query_stats(self._h, C.byref(n)))
        return n.value

    def candidates(self, t: torch.Tensor, m: torch.Tensor):
        i = self.info
        Q = m.shape[0]
        cand = torch.empty((Q, i.n_curves * i.window), dtype=torch.int64, device=t.device)
        nc = torch.empty(Q, dtype=torch.int32, device=t.device)
        _check(_L.sfc_query_candidates(self._h, _ptr(t), _ptr(m), Q, _ptr(cand), _ptr(nc)))
        return cand, nc

    def coords(self, t: torch.Tensor, m: torch.Tensor):
        i = self.info
        Q = m.shape[0]
        sub = torch.empty(Q, dtype=torch.int32, device=t.device)
        y = torch.empty((Q, i.reduced_dim), dtype=torch.float64, device=t.device)
        _check(_L.sfc_query_coords(self._h, _ptr(t), _ptr(m), Q, _ptr(sub), _ptr(y)))
        return sub, y

    def quantized(self) -> torch.Tensor:
        out = torch.empty(self.volume.shape, dtype=torch.uint8, device=self.volume.device)
        _check(_L.sfc_index_quantized(self._h, _ptr(out)))
        return out

    def basis(self, subset: int):
        import numpy as np
        i = self.info
        buf = np.zeros((self.K ** self.mask.dim() * i.channels, i.reduced_dim), np.int8)
        rows = C.c_int32()
        _check(_L.sfc_index_get_basis(self._h, subset, buf.ctypes.data_as(C.c_void_p),
                                      C.byref(rows)))
        return buf[:rows.value].copy()

    def params(self, subset: int):
        import numpy as np
        i = self.info
        lo = np.zeros(i.reduced_dim, np.int64)
        span = C.c_int64()
        _check(_L.sfc_index_get_params(self._h, subset, lo.ctypes.data_as(C.c_void_p),
                                       C.byref(span)))
        return lo, span.value

    def projection(self, subset: int) -> torch.Tensor:
        i = self.info
        y = torch.empty((i.n, i.reduced_dim), dtype=torch.int64, device=self.volume.device)
        _check(_L.sfc_index_projection(self._h, subset, _ptr(y)))
        return y

    def export(self, subset: int, curve: int):
        i = self.info
        keys = torch.empty((i.n, i.key_words), dtype=torch.int64, device=self.volume.device)
        ids = torch.empty(i.n, dtype=torch.int64, device=self.volume.device)
        _check(_L.sfc_index_export(self._h, subset, curve, _ptr(keys), _ptr(ids)))
        return keys, ids


class Batch:
    """Owner of an sfc_batch: many 2D images, one persistent scan launch per
    query, captured in a HIP graph and replayed."""

    def __init__(self, volumes: list, masks: list, K: int, **opts):
        import numpy as np
        self.volumes, self.masks, self.K = list(volumes), list(masks), K
        self._opts = options(**opts)
        n = len(self.volumes)
        vp = (C.c_void_p * n)(*[_ptr(v) for v in self.volumes])
        mp = (C.c_void_p * n)(*[_ptr(m) for m in self.masks])
        geos = (Geometry * n)(*[geometry(m, v.shape[-1]) for v, m in zip(self.volumes, self.masks)])
        h = C.c_void_p()
        _check(_L.sfc_batch_create(n, C.cast(vp, C.c_void_p), C.cast(mp, C.c_void_p),
                                   C.cast(geos, C.c_void_p), K, C.byref(self._opts), C.byref(h)))
        self._h = h
        self._np = np

    def _counts(self, counts):
        arr = self._np.ascontiguousarray(self._np.asarray(counts, dtype=self._np.int64))
        return arr, arr.ctypes.data_as(C.c_void_p)

    def query(self, t: torch.Tensor, m: torch.Tensor, counts, out=None):
        """t: concatenated [count_i, K*K, C_i] float32 (flat is fine); m: [sum, K*K]."""
        arr, cp = self._counts(counts)
        Q = int(arr.sum())
        if out is None:
            out = (torch.empty(Q, dtype=torch.int64, device=m.device),
                   torch.empty(Q, dtype=torch.float32, device=m.device))
        bi, bc = out
        _check(_L.sfc_batch_query(self._h, _ptr(t), _ptr(m), cp, _ptr(bi), _ptr(bc)))
        return bi, bc

    def autotune(self, t: torch.Tensor, m: torch.Tensor, counts, out) -> int:
        arr, cp = self._counts(counts)
        v = C.c_int32()
        bi, bc = out
        _check(_L.sfc_batch_autotune(self._h, _ptr(t), _ptr(m), cp, _ptr(bi), _ptr(bc),
                                     C.byref(v)))
        return v.value

    def stats(self):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int32()
        _check(_L.sfc_batch_stats(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return {"graph_replays": a.value, "work_items": b.value, "shape": c.value}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _L.sfc_batch_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def inpaint(volume: torch.Tensor, mask: torch.Tensor, K: int, order="criminisi", mode="fp32",
            index: Index | None = None, log_cap: int = 0, **opts):
    """Fill in place; returns (iterations, log dict of numpy arrays)."""
    import numpy as np
    o = options(**opts)
    g = geometry(mask, volume.shape[-1])
    n = C.c_int64()
    log = None
    arrs = None
    if log_cap > 0:
        arrs = (np.zeros(log_cap, np.int64), np.zeros(log_cap, np.int64),
                np.zeros(log_cap, np.float32))
        log = FillLog()
        log.cap = log_cap
        log.centre_host = arrs[0].ctypes.data
        log.source_host = arrs[1].ctypes.data
        log.cost_host = arrs[2].ctypes.data
    _check(_L.sfc_inpaint(_ptr(volume), _ptr(mask), C.byref(g), K, ORDERS[order], MODES[mode],
                          index._h if index is not None else None, C.byref(o), C.byref(n),
                          C.byref(log) if log is not None else None))
    out = {}
    if arrs is not None:
        k = min(log.len, log_cap)
        out = dict(centre=arrs[0][:k].copy(), source=arrs[1][:k].copy(), cost=arrs[2][:k].copy())
    return n.value, out
