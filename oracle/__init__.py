"""CPU oracle for the masked-L2 patch search (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. It wraps the plain single-threaded C implementation in
`oracle.c` (built with gcc, no fused operations) and composes its steps in the
order the paper gives them. It shares no code with the GPU library and never
takes an input from it.

Functions return numpy arrays; inputs are numpy arrays laid out as documented
in `oracle.c`.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
GCC_FLAGS = ["-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC"]

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc; returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *GCC_FLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = _declare(C.CDLL(_LIB))
    return _lib


P = C.c_void_p
I64 = C.c_int64
I32 = C.c_int


class OrcIndex(C.Structure):
    _fields_ = [
        ("nd", C.c_int), ("shape", C.c_int64 * 3),
        ("C", C.c_int), ("K", C.c_int), ("S", C.c_int), ("D", C.c_int), ("L", C.c_int),
        ("b", C.c_int), ("curve", C.c_int), ("window", C.c_int),
        ("n", C.c_int64), ("dict", P), ("vmin", C.c_float), ("qscale", C.c_float),
        ("npix", P), ("pix", P), ("basis", P), ("basis_off", P), ("lo", P), ("span", P),
        ("sum", P), ("nsub", C.c_int64), ("keys", P), ("ids", P), ("norm", C.c_int),
    ]


def _declare(L):
    sig = {
        "orc_front": (I64, [P, I32, P, P, I64]),
        "orc_priority": (None, [P, P, P, I32, P, I32, I32, I64, P, P]),
        "orc_extract": (None, [P, P, I32, P, I32, I32, P, I64, P, P]),
        "orc_dictionary": (I64, [P, I32, P, I32, P, I64]),
        "orc_cost_one": (C.c_float, [P, I32, P, I32, I32, I64, P, P]),
        "orc_cost64_one": (C.c_double, [P, I32, P, I32, I32, I64, P, P]),
        "orc_cost_l1_one": (C.c_float, [P, I32, P, I32, I32, I64, P, P]),
        "orc_cost64_l1_one": (C.c_double, [P, I32, P, I32, I32, I64, P, P]),
        "orc_brute": (None, [P, I32, P, I32, I32, P, I64, P, P, I64, P, P, I32]),
        "orc_quantize": (I32, [P, P, I64, I32, P, P, P]),
        "orc_subsets": (I32, [I32, I32, P, P]),
        "orc_cov_sums": (I64, [P, I32, P, I32, I32, P, I64, P, P]),
        "orc_cov_matrix": (None, [P, P, I64, I64, P, I32, P]),
        "orc_jacobi": (I32, [P, I32, P]),
        "orc_basis": (I32, [P, P, I32, I32, P, P]),
        "orc_project": (None, [P, I32, P, I32, I32, P, I64, P, I32, P, I32, P]),
        "orc_key_params": (None, [P, I64, I32, P, P]),
        "orc_key_of": (None, [P, I32, I32, I32, P]),
        "orc_keys": (None, [P, I64, I32, P, I64, I32, I32, I32, I32, P]),
        "orc_sort": (None, [P, P, I64, I32]),
        "orc_query": (None, [C.POINTER(OrcIndex), P, P, P, I64, P, P, P, P, P]),
        "orc_knn": (I32, [C.POINTER(OrcIndex), P, P, P, I64, I32, P, P, P, P]),
        "orc_morton_decode": (None, [P, I32, I32, P]),
        "orc_query_point": (I32, [C.POINTER(OrcIndex), P, P, P]),
        "orc_choose_subset": (I32, [P, P, I32, I64, P]),
        "orc_window": (I64, [P, I64, I32, P, I32, P]),
        "orc_inpaint": (I64, [P, P, I32, P, I32, I32, I32, I32, P, I64,
                              C.POINTER(OrcIndex), I64, P, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _shape(shape):
    s = np.zeros(3, dtype=np.int64)
    s[:len(shape)] = shape
    return s


# ---------------------------------------------------------------- basics
def priority(volume, mask, K, p, conf=None):
    """(P, C_p) of front voxel p (flat id) in the fill order's reading;
    conf defaults to 1 on known voxels and 0 elsewhere (the first step)."""
    volume, mask = _c(volume, np.float32), _c(mask, np.uint8)
    if conf is None:
        conf = (mask != 0).astype(np.float64)
    conf = _c(conf, np.float64)
    P_, C_ = C.c_double(), C.c_double()
    lib().orc_priority(_p(volume), _p(mask), _p(conf), mask.ndim, _p(_shape(mask.shape)),
                       volume.shape[-1], K, int(p), C.byref(P_), C.byref(C_))
    return P_.value, C_.value


def front(mask):
    mask = _c(mask, np.uint8)
    out = np.empty(mask.size, dtype=np.int64)
    n = lib().orc_front(_p(mask), mask.ndim, _p(_shape(mask.shape)), _p(out), out.size)
    return out[:n].copy()


def extract(volume, mask, K, centres):
    volume, mask = _c(volume, np.float32), _c(mask, np.uint8)
    nd, Cc = mask.ndim, volume.shape[-1]
    centres = _c(centres, np.int64)
    Q, Kd = centres.size, K ** nd
    t = np.empty((Q, Kd, Cc), dtype=np.float32)
    m = np.empty((Q, Kd), dtype=np.uint8)
    lib().orc_extract(_p(volume), _p(mask), nd, _p(_shape(mask.shape)), Cc, K,
                      _p(centres), Q, _p(t), _p(m))
    return t, m


def dictionary(mask, K):
    mask = _c(mask, np.uint8)
    out = np.empty(mask.size, dtype=np.int64)
    n = lib().orc_dictionary(_p(mask), mask.ndim, _p(_shape(mask.shape)), K, _p(out), out.size)
    return out[:n].copy()


def dictionary_pooled(mask, K, threads):
    """dictionary() computed over slabs of the slowest axis in a thread pool:
    the slab of centre rows [a, b) with h = (K-1)/2 rows of halo on each side
    (clipped to the volume) holds every box of those centres, so the oracle's
    dictionary of the slab, restricted to rows [a, b) and offset back, is the
    full dictionary's part for those rows."""
    mask = _c(mask, np.uint8)
    if threads <= 1 or mask.shape[0] < 4 * threads:
        return dictionary(mask, K)
    h = (K - 1) // 2
    row = int(np.prod(mask.shape[1:]))
    cuts = np.linspace(0, mask.shape[0], 2 * threads + 1).astype(int)

    def part(ab):
        a, b = ab
        lo, hi = max(0, a - h), min(mask.shape[0], b + h)
        ids = dictionary(mask[lo:hi], K)
        r = ids // row + lo
        return ids[(r >= a) & (r < b)] + lo * row

    parts = _pool_map(part, [(int(a), int(b)) for a, b in zip(cuts[:-1], cuts[1:]) if b > a],
                      threads)
    return np.concatenate(parts)


NORMS = {"l2": 0, "l1": 1}


def cost(volume, shape, K, centre, t, m, norm="l2"):
    """The float32 cost that ranks candidates: masked L2 (Section II) or the
    L1 variant of Section III.K."""
    volume = _c(volume, np.float32)
    t, m = _c(t, np.float32), _c(m, np.uint8)
    f = lib().orc_cost_l1_one if NORMS[norm] else lib().orc_cost_one
    return float(f(_p(volume), len(shape), _p(_shape(shape)), volume.shape[-1], K, int(centre),
                   _p(t), _p(m)))


def cost64(volume, shape, K, centre, t, m, norm="l2"):
    volume = _c(volume, np.float32)
    t, m = _c(t, np.float32), _c(m, np.uint8)
    f = lib().orc_cost64_l1_one if NORMS[norm] else lib().orc_cost64_one
    return float(f(_p(volume), len(shape), _p(_shape(shape)), volume.shape[-1], K, int(centre),
                   _p(t), _p(m)))


def brute(volume, shape, K, dict_ids, t, m, norm="l2"):
    volume = _c(volume, np.float32)
    dict_ids = _c(dict_ids, np.int64)
    t, m = _c(t, np.float32), _c(m, np.uint8)
    Q = m.shape[0]
    bi = np.empty(Q, dtype=np.int64)
    bc = np.empty(Q, dtype=np.float32)
    lib().orc_brute(_p(volume), len(shape), _p(_shape(shape)), volume.shape[-1], K,
                    _p(dict_ids), dict_ids.size, _p(t), _p(m), Q, _p(bi), _p(bc), NORMS[norm])
    return bi, bc


def brute_pooled(volume, shape, K, dict_ids, t, m, threads, norm="l2"):
    """brute() over slices of the dictionary in a thread pool, merged by
    (cost, id): slices ascend, so on equal costs the earlier slice's (lower)
    id stays, as in one full scan."""
    dict_ids = _c(dict_ids, np.int64)
    parts = _pool_map(lambda d: brute(volume, shape, K, d, t, m, norm),
                      [x for x in np.array_split(dict_ids, max(1, 2 * threads)) if x.size],
                      threads)
    bi, bc = parts[0][0].copy(), parts[0][1].copy()
    for pi, pc in parts[1:]:
        take = pc < bc
        bi[take], bc[take] = pi[take], pc[take]
    return bi, bc


# ---------------------------------------------------------------- index build steps
def quantize(volume, mask):
    volume, mask = _c(volume, np.float32), _c(mask, np.uint8)
    xq = np.empty(volume.shape, dtype=np.uint8)
    vmin = C.c_float()
    sc = C.c_float()
    rc = lib().orc_quantize(_p(volume), _p(mask), mask.size, volume.shape[-1],
                            C.byref(vmin), C.byref(sc), _p(xq))
    if rc != 0:
        raise ValueError("no known voxel")
    return xq, np.float32(vmin.value), np.float32(sc.value)


def subsets(nd, K):
    Kd = K ** nd
    S_max = 3 ** nd - 1
    npix = np.empty(S_max, dtype=np.int32)
    pix = np.full((S_max, Kd), -1, dtype=np.int32)
    S = lib().orc_subsets(nd, K, _p(npix), _p(pix))
    return [pix[s, :npix[s]].copy() for s in range(S)]


def subset_elems(pix, Cc):
    return (np.repeat(pix.astype(np.int64) * Cc, Cc) + np.tile(np.arange(Cc), pix.size)).astype(np.int32)


def cov_sums(xq, shape, K, dict_ids):
    xq = _c(xq, np.uint8)
    Cc = xq.shape[-1]
    P = K ** len(shape) * Cc
    dict_ids = _c(dict_ids, np.int64)
    s = np.empty(P, dtype=np.int64)
    ss = np.empty((P, P), dtype=np.int64)
    nsub = lib().orc_cov_sums(_p(xq), len(shape), _p(_shape(shape)), Cc, K,
                              _p(dict_ids), dict_ids.size, _p(s), _p(ss))
    return s, ss, int(nsub)


def _pool_map(fn, items, threads):
    if threads <= 1:
        return [fn(x) for x in items]
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(threads) as ex:   # ctypes releases the GIL during each call
        return list(ex.map(fn, items))


def cov_sums_pooled(xq, shape, K, dict_ids, threads):
    """cov_sums over the same strided subsample, computed as exact integer
    sums over slices of it in a thread pool (each slice holds under 2^20
    ranks, so orc_cov_sums takes every rank of a slice)."""
    dict_ids = _c(dict_ids, np.int64)
    stride = max(1, -(-dict_ids.size // (1 << 20)))
    sub = dict_ids[::stride]
    parts = _pool_map(lambda d: cov_sums(xq, shape, K, d),
                      [x for x in np.array_split(sub, max(1, 2 * threads)) if x.size], threads)
    s = sum(p[0] for p in parts)
    ss = sum(p[1] for p in parts)
    assert sum(p[2] for p in parts) == sub.size
    return s, ss, int(sub.size)


def cov_matrix(s, ss, nsub, elems):
    elems = _c(elems, np.int32)
    m = elems.size
    A = np.empty((m, m), dtype=np.float64)
    lib().orc_cov_matrix(_p(s), _p(_c(ss, np.int64)), nsub, s.size, _p(elems), m, _p(A))
    return A


def jacobi(A):
    A = np.array(A, dtype=np.float64, order="C", copy=True)
    m = A.shape[0]
    V = np.empty((m, m), dtype=np.float64)
    sweeps = lib().orc_jacobi(_p(A), m, _p(V))
    return A, V, int(sweeps)


def basis_from(A_diag_form, V, D):
    A_diag_form = _c(A_diag_form, np.float64)
    V = _c(V, np.float64)
    m = V.shape[0]
    w = np.empty((m, D), dtype=np.int8)
    order = np.empty(D, dtype=np.int32)
    if lib().orc_basis(_p(A_diag_form), _p(V), m, D, _p(w), _p(order)) != 0:
        raise ValueError("reduced dimension out of range")
    return w, order


def project(xq, shape, K, dict_ids, elems, w):
    xq = _c(xq, np.uint8)
    dict_ids, elems, w = _c(dict_ids, np.int64), _c(elems, np.int32), _c(w, np.int8)
    D = w.shape[1]
    y = np.empty((dict_ids.size, D), dtype=np.int64)
    lib().orc_project(_p(xq), len(shape), _p(_shape(shape)), xq.shape[-1], K, _p(dict_ids),
                      dict_ids.size, _p(elems), elems.size, _p(w), D, _p(y))
    return y


def key_params(y):
    y = _c(y, np.int64)
    n, D = y.shape
    lo = np.empty(D, dtype=np.int64)
    span = C.c_int64()
    lib().orc_key_params(_p(y), n, D, _p(lo), C.byref(span))
    return lo, int(span.value)


def key_words(D, b):
    return (D * b + 63) // 64


def key_of(v, b, curve):
    v = _c(v, np.uint32)
    D = v.size
    out = np.zeros(key_words(D, b), dtype=np.uint64)
    lib().orc_key_of(_p(v), D, b, curve, _p(out))
    return out


def keys(y, lo, span, b, j, L, curve):
    y, lo = _c(y, np.int64), _c(lo, np.int64)
    n, D = y.shape
    out = np.empty((n, key_words(D, b)), dtype=np.uint64)
    lib().orc_keys(_p(y), n, D, _p(lo), span, b, j, L, curve, _p(out))
    return out


def sort(keys_, ids):
    keys_ = np.array(keys_, dtype=np.uint64, order="C", copy=True)
    ids = np.array(ids, dtype=np.int64, order="C", copy=True)
    lib().orc_sort(_p(keys_), _p(ids), ids.size, keys_.shape[1] if keys_.ndim == 2 else 1)
    return keys_, ids


def choose_subset(pix, m):
    """The query's subset (Fig. 1b) for target pixel mask m [K^nd]: pix is the
    list of subsets (pixel offsets), as subsets() returns it."""
    m = _c(m, np.uint8)
    Kd = m.size
    npix = np.array([p.size for p in pix], dtype=np.int32)
    pixa = np.full((len(pix), Kd), -1, dtype=np.int32)
    for s, p in enumerate(pix):
        pixa[s, :p.size] = p
    return int(lib().orc_choose_subset(_p(npix), _p(pixa), len(pix), Kd, _p(m)))


def window(sorted_keys, qkey, W):
    """(p, lo) of the candidate window of width W on one sorted curve for the
    query key qkey (uint64 words, word 0 most significant)."""
    k = _c(sorted_keys, np.uint64)
    if k.ndim == 1:
        k = k.reshape(-1, 1)
    qk = _c(np.atleast_1d(np.asarray(qkey, dtype=np.uint64)), np.uint64)
    assert qk.size == k.shape[1]
    p = C.c_int64()
    lo = lib().orc_window(_p(k), k.shape[0], k.shape[1], _p(qk), int(W), C.byref(p))
    return int(p.value), int(lo)


CURVES = {"morton": 0, "hilbert": 1}


class Index:
    """The SFC multi-index built by the oracle's steps, in the paper's order:
    byte quantisation, pixel subsets, PCA to D dims, grid cell on L shifted
    curves, sort by curve position (Sections II, II.A-C)."""

    def __init__(self, volume, mask, K, D, L, key_bits=8, curve="morton", window=32,
                 bases=None, keep_y=False, norm="l2", threads=1, build_curves=True):
        """threads > 1 runs independent oracle calls (slices of the covariance
        subsample, separate subsets) in a thread pool; the result is the same.
        build_curves=False stops after the statistics and bases: curves are
        then attached one by one with attach_curve()."""
        self.volume = _c(volume, np.float32)
        self.mask = _c(mask, np.uint8)
        self.shape = tuple(self.mask.shape)
        self.nd = len(self.shape)
        self.C = self.volume.shape[-1]
        self.K, self.D, self.L, self.b, self.window = K, D, L, key_bits, window
        self.norm = NORMS[norm]   # the rescoring cost (the index itself is norm-free)
        self.curve = CURVES[curve] if isinstance(curve, str) else int(curve)
        self.xq, self.vmin, self.qscale = quantize(self.volume, self.mask)
        self.dict = dictionary_pooled(self.mask, K, threads)
        self.n = self.dict.size
        if self.n == 0:
            raise ValueError("empty dictionary")
        self.pix = subsets(self.nd, K)
        self.S = len(self.pix)
        self.elems = [subset_elems(p, self.C) for p in self.pix]
        if threads > 1:
            self.sum, self.sumsq, self.nsub = cov_sums_pooled(self.xq, self.shape, K, self.dict,
                                                              threads)
        else:
            self.sum, self.sumsq, self.nsub = cov_sums(self.xq, self.shape, K, self.dict)
        self.W64 = key_words(D, key_bits)
        self.y = [None] * self.S if keep_y else None
        self.sweeps = [None] * self.S

        def basis_of(s):
            if bases is not None:
                return _c(bases[s], np.int8)
            A = cov_matrix(self.sum, self.sumsq, self.nsub, self.elems[s])
            Ad, V, sw = jacobi(A)
            self.sweeps[s] = sw
            return basis_from(Ad, V, D)[0]

        self.bases = _pool_map(basis_of, range(self.S), threads)
        self.lo, self.span = [None] * self.S, [None] * self.S
        self._curves = {}
        if not build_curves:
            self.keys = self.ids = None
            self._struct = None
            return
        self.keys = np.empty((self.S, L, self.n, self.W64), dtype=np.uint64)
        self.ids = np.empty((self.S, L, self.n), dtype=np.int64)

        def subset_curves(s):
            y = project(self.xq, self.shape, K, self.dict, self.elems[s], self.bases[s])
            if keep_y:
                self.y[s] = y
            lo, span = key_params(y)
            self.lo[s], self.span[s] = lo, span
            for j in range(L):
                k = keys(y, lo, span, key_bits, j, L, self.curve)
                k, i = sort(k, self.dict)
                self.keys[s, j] = k
                self.ids[s, j] = i

        _pool_map(subset_curves, range(self.S), threads)
        for s in range(self.S):
            for j in range(L):
                self._curves[(s, j)] = (self.keys[s, j], self.ids[s, j])
        self._struct = None

    def attach_curve(self, s, j, lo, span, sorted_keys, sorted_ids):
        """Attach one sorted curve of subset s (grid origin lo, span) to an
        index built with build_curves=False. The caller must have shown the
        arrays to be this index's own: strictly increasing in (key, id), a
        permutation of the dictionary, and every key equal to the key this
        oracle computes for that id; sorting is then unique, so they equal
        what sort() would return."""
        k = _c(sorted_keys, np.uint64).reshape(self.n, self.W64)
        i = _c(sorted_ids, np.int64)
        assert i.size == self.n
        self.lo[s], self.span[s] = _c(lo, np.int64), int(span)
        self._curves[(s, j)] = (k, i)
        self._struct = None

    def drop_curves(self):
        self._curves = {}
        self._struct = None

    def struct(self):
        if self._struct is None:
            Kd = self.K ** self.nd
            self._npix = np.array([p.size for p in self.pix], dtype=np.int32)
            self._pixa = np.full((self.S, Kd), -1, dtype=np.int32)
            for s, p in enumerate(self.pix):
                self._pixa[s, :p.size] = p
            self._basis = np.concatenate([w.ravel() for w in self.bases]).astype(np.int8)
            self._boff = np.cumsum([0] + [w.size for w in self.bases[:-1]]).astype(np.int64)
            self._lo = np.zeros((self.S, self.D), dtype=np.int64)
            self._span = np.ones(self.S, dtype=np.int64)
            for s_ in range(self.S):
                if self.lo[s_] is not None:
                    self._lo[s_] = self.lo[s_]
                    self._span[s_] = self.span[s_]
            nc = self.S * self.L
            self._kp = (C.c_void_p * nc)()
            self._ip = (C.c_void_p * nc)()
            for (s_, j), (k, i) in self._curves.items():
                self._kp[s_ * self.L + j] = k.ctypes.data
                self._ip[s_ * self.L + j] = i.ctypes.data
            st = OrcIndex()
            st.nd = self.nd
            for i, v in enumerate(self.shape):
                st.shape[i] = v
            st.C, st.K, st.S, st.D, st.L = self.C, self.K, self.S, self.D, self.L
            st.b, st.curve, st.window, st.n = self.b, self.curve, self.window, self.n
            st.dict = _p(self.dict)
            st.vmin, st.qscale = float(self.vmin), float(self.qscale)
            st.npix, st.pix = _p(self._npix), _p(self._pixa)
            st.basis, st.basis_off = _p(self._basis), _p(self._boff)
            st.lo, st.span = _p(self._lo), _p(self._span)
            st.sum, st.nsub = _p(self.sum), self.nsub
            st.keys = C.cast(self._kp, C.c_void_p)
            st.ids = C.cast(self._ip, C.c_void_p)
            st.norm = self.norm
            self._struct = st
        return self._struct

    def query_point(self, t, m):
        """Subset choice and real principal coordinates of each query."""
        t, m = _c(t, np.float32), _c(m, np.uint8)
        Q = m.shape[0]
        sub = np.empty(Q, dtype=np.int32)
        ys = np.empty((Q, self.D), dtype=np.float64)
        buf = np.empty(64, dtype=np.float64)
        st = C.byref(self.struct())
        for q in range(Q):
            sub[q] = lib().orc_query_point(st, _p(t[q]), _p(m[q]), _p(buf))
            ys[q] = buf[:self.D]
        return sub, ys

    def _check_curves(self, m, curves):
        """Every query's subset must have the curves the query reads."""
        if len(self._curves) == self.S * self.L:
            return
        for q in range(m.shape[0]):
            s = choose_subset(self.pix, m[q])
            for j in curves:
                if (s, j) not in self._curves:
                    raise ValueError(f"query {q} needs curve ({s}, {j}), which is not attached")

    def query(self, volume, t, m):
        """Returns (best_id, best_cost, candidates [Q, L*W] padded -1,
        ncand [Q], subset [Q])."""
        volume = _c(volume, np.float32)
        t, m = _c(t, np.float32), _c(m, np.uint8)
        self._check_curves(m, range(self.L))
        Q = m.shape[0]
        cap = self.L * self.window
        bi = np.empty(Q, dtype=np.int64)
        bc = np.empty(Q, dtype=np.float32)
        cand = np.empty((Q, cap), dtype=np.int64)
        nc = np.empty(Q, dtype=np.int32)
        sub = np.empty(Q, dtype=np.int32)
        lib().orc_query(C.byref(self.struct()), _p(volume), _p(t), _p(m), Q, _p(bi), _p(bc),
                        _p(cand), _p(nc), _p(sub))
        return bi, bc, cand, nc, sub

    def knn_query(self, volume, t, m, k=80):
        """Exact k-NN query of Section II.D on the unshifted Morton curve.
        Returns (best_id, best_cost, candidates [Q, k] ascending ids padded
        -1, ncand [Q])."""
        volume = _c(volume, np.float32)
        t, m = _c(t, np.float32), _c(m, np.uint8)
        self._check_curves(m, [0])
        Q = m.shape[0]
        bi = np.empty(Q, dtype=np.int64)
        bc = np.empty(Q, dtype=np.float32)
        cand = np.empty((Q, k), dtype=np.int64)
        nc = np.empty(Q, dtype=np.int32)
        r = lib().orc_knn(C.byref(self.struct()), _p(volume), _p(t), _p(m), Q, k, _p(bi), _p(bc),
                          _p(cand), _p(nc))
        if r != 0:
            raise ValueError("k-NN needs a Morton-ordered index, k >= 1 and "
                             "2*key_bits + ceil(log2(D)) <= 62")
        return bi, bc, cand, nc


def morton_decode(key_words, D, b):
    """Coordinates [D] (uint32) of one Morton key (uint64 words, word 0 most
    significant)."""
    kw = _c(np.asarray(key_words, dtype=np.uint64), np.uint64)
    v = np.empty(D, dtype=np.uint32)
    lib().orc_morton_decode(_p(kw), D, b, _p(v))
    return v


def inpaint(volume, mask, K, order="criminisi", mode="brute", index: Index | None = None,
            cap=None):
    """Runs the fill loop on copies; returns (volume, mask, log dict)."""
    vol = np.array(volume, dtype=np.float32, order="C", copy=True)
    msk = np.array(mask, dtype=np.uint8, order="C", copy=True)
    shape = msk.shape
    d = dictionary(msk, K)
    cap = int(msk.size if cap is None else cap)
    lc = np.empty(cap, dtype=np.int64)
    ls = np.empty(cap, dtype=np.int64)
    lcost = np.empty(cap, dtype=np.float32)
    o = {"criminisi": 0, "raster": 1}[order]
    md = {"brute": 0, "index": 3}[mode]
    ixp = C.byref(index.struct()) if (md == 3 and index is not None) else None
    it = lib().orc_inpaint(_p(vol), _p(msk), len(shape), _p(_shape(shape)), vol.shape[-1], K,
                           o, md, _p(d), d.size, ixp, cap, _p(lc), _p(ls), _p(lcost))
    if it < 0:
        raise RuntimeError("inpaint failed with code %d" % it)
    k = min(int(it), cap)
    return vol, msk, dict(iters=int(it), centre=lc[:k].copy(), source=ls[:k].copy(),
                          cost=lcost[:k].copy())
