"""GPU parity at full size: the 256^3 tomogram (n ~ 1.4e7, 7^3 patches, 6
Hilbert curves, two-word keys) and the 512^3 phantom (n ~ 1.25e8, 5^3 patches,
4 Morton curves, one-word keys), built in the same launch configuration the
benchmark times.

At these sizes the oracle cannot build the whole index, so the checks are the
outputs it can compute one by one and properties that hold at any size:
  - dictionary: equal to the interior erosion of the mask;
  - bases: equal to the oracle's, from the same exact covariance sums;
  - one subset's projections: sampled rows equal the oracle's, and the grid
    origin and span are their column minima and largest range;
  - that subset's sorted curves: strictly increasing in (key, id), a
    permutation of the dictionary, and sampled keys equal the oracle's keys
    of the oracle's projections;
  - queries: the float32 scan equals the oracle's full scan on sampled
    targets, every returned cost equals the oracle's cost of the returned id,
    the index never beats the scan, and the bf16 scan equals the float32 scan.
The oracle is single-threaded; the tests run independent oracle calls (slices
of the dictionary or of the covariance subsample, separate subsets) in a
thread pool and merge them exactly: the minimum over (cost, id) is
associative, and integer sums are exact.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
from scipy.ndimage import minimum_filter

import oracle
from paper_1712_06326_amd import synth

from gpu_util import dev, host, need_gpu, say

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, os.cpu_count() or 1))


def _pool_map(fn, items):
    with ThreadPoolExecutor(THREADS) as ex:
        return list(ex.map(fn, items))


def _brute_parallel(vol, shape, K, dict_ids, t, m):
    """The oracle's full scan over dictionary slices, merged by (cost, id)."""
    slices = np.array_split(dict_ids, THREADS * 2)
    parts = _pool_map(lambda d: oracle.brute(vol, shape, K, d, t, m), [s for s in slices if s.size])
    bi, bc = parts[0][0].copy(), parts[0][1].copy()
    for pi, pc in parts[1:]:   # slices ascend, so a tie keeps the earlier (lower) id
        take = pc < bc
        bi[take], bc[take] = pi[take], pc[take]
    return bi, bc


def _cov_sums_parallel(xq, shape, K, dict_ids):
    """The oracle's covariance sums over the strided subsample, summed over
    slices of it (each slice is under 2^20 ranks, so no further stride)."""
    stride = max(1, -(-dict_ids.size // (1 << 20)))
    sub = dict_ids[::stride]
    parts = _pool_map(lambda d: oracle.cov_sums(xq, shape, K, d),
                      [s for s in np.array_split(sub, THREADS * 2) if s.size])
    s = sum(p[0] for p in parts)
    ss = sum(p[1] for p in parts)
    assert sum(p[2] for p in parts) == sub.size
    return s, ss, sub.size


def _increasing(keys, ids):
    """(key words, id) strictly increasing along the array."""
    keys = keys.reshape(keys.shape[0], -1)
    gt = np.zeros(keys.shape[0] - 1, dtype=bool)
    eq = np.ones(keys.shape[0] - 1, dtype=bool)
    for w in range(keys.shape[1]):
        a, b = keys[:-1, w], keys[1:, w]
        gt |= eq & (b > a)
        eq &= b == a
    gt |= eq & (ids[1:] > ids[:-1])
    return bool(np.all(gt))


def _run(name, n_queries, n_brute, check_bf16, curves_checked):
    nat = need_gpu()
    d = getattr(synth, name)()
    vol, mask, K = d["volume"], d["mask"], d["K"]
    D, L, b, curve, W = d["D"], d["n_curves"], d["key_bits"], d["curve"], d["window"]
    say(f"{name}: {mask.shape} K={K} D={D} L={L} b={b} {curve} W={W}")
    vd, md = dev(vol), dev(mask)
    ix = nat.Index(vd, md, K, reduced_dim=D, n_curves=L, key_bits=b, window=W, curve=curve)
    info = ix.info
    say(f"  built: n={info.n}")

    # dictionary = interior erosion of the mask
    er = minimum_filter(mask, size=K, mode="constant", cval=0)
    dict_ids = np.flatnonzero(er).astype(np.int64)
    assert info.n == dict_ids.size
    assert np.array_equal(host(ix.dictionary()), dict_ids)
    say("  dictionary ok")

    # bases from the oracle's own covariance, eigensolver and rounding
    xq, vmin, qs = oracle.quantize(vol, mask)
    assert np.float32(info.vmin) == vmin and np.float32(info.qscale) == qs
    s_, ss_, nsub = _cov_sums_parallel(xq, mask.shape, K, dict_ids)
    assert info.n_sub == nsub
    pix = oracle.subsets(mask.ndim, K)
    elems = [oracle.subset_elems(p, vol.shape[-1]) for p in pix]

    def basis_of(e):
        A, V, _ = oracle.jacobi(oracle.cov_matrix(s_, ss_, nsub, e))
        return oracle.basis_from(A, V, D)[0]

    bases = _pool_map(basis_of, elems)
    for s in range(len(pix)):
        assert np.array_equal(ix.basis(s), bases[s]), f"basis of subset {s}"
    say(f"  {len(pix)} bases ok")

    # one subset: projections, grid, sorted curves
    rng = np.random.default_rng(123)
    s = len(pix) - 1
    y = host(ix.projection(s))
    lo, span = ix.params(s)
    rows = np.sort(rng.choice(info.n, 20000, replace=False))
    yo = oracle.project(xq, mask.shape, K, dict_ids[rows], elems[s], bases[s])
    assert np.array_equal(y[rows], yo)
    assert np.array_equal(lo, y.min(axis=0))
    assert span == max(1, int((y.max(axis=0) - lo).max()))
    del y
    say(f"  projection and grid of subset {s} ok")
    seen = np.zeros(mask.size, dtype=bool)
    for j in curves_checked:
        k_, i_ = ix.export(s, j)
        keys, ids = host(k_).view(np.uint64).reshape(info.n, -1), host(i_)
        del k_, i_
        assert _increasing(keys, ids), f"curve ({s},{j}) not sorted by (key, id)"
        seen[:] = False
        seen[ids] = True
        assert np.count_nonzero(seen) == info.n and np.array_equal(np.flatnonzero(seen), dict_ids)
        pos = np.sort(rng.choice(info.n, 4096, replace=False))
        yp = oracle.project(xq, mask.shape, K, ids[pos], elems[s], bases[s])
        ko = oracle.keys(yp, lo, span, b, j, L, oracle.CURVES[curve])
        assert np.array_equal(keys[pos], ko.reshape(pos.size, -1)), f"keys of curve ({s},{j})"
        say(f"  curve ({s},{j}) ok")
    del seen

    # queries on a seeded sample of the front
    f = oracle.front(mask)
    sel = np.sort(rng.choice(f.size, n_queries, replace=False))
    t, m = oracle.extract(vol, mask, K, f[sel])
    td, mq = dev(t), dev(m)
    bs, cs = (host(a) for a in ix.query(td, mq, "fp32"))
    bx, cx = (host(a) for a in ix.query(td, mq, "index"))
    for q in range(n_queries):
        assert np.float32(oracle.cost(vol, mask.shape, K, bs[q], t[q], m[q])).view(np.uint32) == \
            cs[q].view(np.uint32)
        assert np.float32(oracle.cost(vol, mask.shape, K, bx[q], t[q], m[q])).view(np.uint32) == \
            cx[q].view(np.uint32)
    assert np.all(cx >= cs)
    assert np.all(er.ravel()[bs] != 0) and np.all(er.ravel()[bx] != 0)
    say(f"  {n_queries} sampled queries: costs of returned ids ok")
    ob, oc = _brute_parallel(vol, mask.shape, K, dict_ids, t[:n_brute], m[:n_brute])
    assert np.array_equal(ob, bs[:n_brute])
    assert np.array_equal(oc.view(np.uint32), cs[:n_brute].view(np.uint32))
    say(f"  float32 scan equals the oracle's full scan on {n_brute} queries")
    if check_bf16:
        br, cr = (host(a) for a in ix.query(td, mq, "bf16"))
        assert np.array_equal(br, bs) and np.array_equal(cr.view(np.uint32), cs.view(np.uint32))
        say(f"  bf16 scan equals the float32 scan ({ix.fallbacks()} fallbacks)")
    ix.close()


def test_scale_tomogram_256cube():
    _run("config3", n_queries=256, n_brute=4, check_bf16=True, curves_checked=(0, 5))


def test_scale_phantom_512cube():
    _run("config4", n_queries=64, n_brute=2, check_bf16=False, curves_checked=(0, 3))
