"""GPU parity at full size: the 1024^2 RGB image (n ~ 0.9e6, 9x9x3 patches,
4 Morton curves, three-word keys), the 256^3 tomogram (n ~ 1.4e7, 7^3
patches, 6 Hilbert curves, two-word keys) and the 512^3 phantom
(n ~ 1.25e8, 5^3 patches, 4 Morton curves, one-word keys), each built in the
launch configuration the benchmark times.

1024^2 RGB: the oracle builds the whole index itself (independent subsets in
a thread pool) and every stage is compared with the GPU's: bases, grids,
projections, all 32 sorted curves; then 256 seeded front queries are
compared in subset, candidate set, selected id and cost bits, and 512 seeded
front queries of the float32 scan against the oracle's full scan.

256^3 and 512^3: the oracle cannot sort curves of 1.4e7-1.25e8 entries in
test time, so:
  - dictionary: equal to the interior erosion of the mask and the oracle's;
  - bases: equal to the oracle's, from the same exact covariance sums;
  - for the subsets that the sampled index queries choose: the oracle's full
    projection (equal to the GPU's for the first of them), its grid (equal to
    the GPU's), and every curve of the subset verified against the oracle's
    keys: the GPU's array is strictly increasing in (key, id), a permutation
    of the dictionary, and every entry's key equals the key the oracle
    computes for that id. Sorting by (key, id) with unique ids has one
    result, so the verified array is the oracle's sorted curve; the oracle's
    query routine then answers the sampled queries on it, and subsets,
    candidate sets, ids and cost bits are compared with the GPU's;
  - the float32 scan equals the oracle's full scan on 32 sampled targets;
    every returned cost equals the oracle's cost of the returned id; the
    index never beats the scan; the bf16 scan equals the float32 scan.
The oracle is single-threaded; independent oracle calls (slices of the
dictionary, of the covariance subsample, separate subsets) run in a thread
pool and are merged exactly: the minimum over (cost, id) is associative,
integer sums are exact, and concatenated slices are the whole array.
"""
import os
from collections import Counter
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
    return oracle.brute_pooled(vol, shape, K, dict_ids, t, m, THREADS)


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


def _slices(n):
    return [s for s in np.array_split(np.arange(n), THREADS * 4) if s.size]


def _compare_queries(ix, ox, vol, t, m, tag):
    """Subset, candidate set, selected id and cost bits of the index query
    against the oracle's query routine."""
    td, mq = dev(t), dev(m)
    sub, _ = ix.coords(td, mq)
    cand, nc = ix.candidates(td, mq)
    bi, bc = ix.query(td, mq, "index")
    bo, co, cando, nco, so = ox.query(vol, t, m)
    assert np.array_equal(host(sub), so), f"{tag}: subsets"
    assert np.array_equal(host(nc), nco), f"{tag}: candidate counts"
    assert np.array_equal(host(cand), cando), f"{tag}: candidate sets"
    assert np.array_equal(host(bi), bo), f"{tag}: selected ids"
    assert np.array_equal(host(bc).view(np.uint32), co.view(np.uint32)), f"{tag}: cost bits"
    say(f"  {tag}: {len(bo)} index queries equal the oracle's (subsets {sorted(set(so.tolist()))})")
    return host(bi), host(bc)


def test_index_config2_full_parity():
    """1024^2 RGB, n ~ 0.9e6: the whole index built by the oracle, every
    stage and 256 index queries compared; 512 float32-scan queries."""
    nat = need_gpu()
    d = synth.config2()
    vol, mask, K = d["volume"], d["mask"], d["K"]
    D, L, b, curve, W = d["D"], d["n_curves"], d["key_bits"], d["curve"], d["window"]
    say(f"config2 index parity: {mask.shape}x{vol.shape[-1]} K={K} D={D} L={L} b={b} W={W}")
    ox = oracle.Index(vol, mask, K, D, L, key_bits=b, curve=curve, window=W, threads=THREADS,
                      keep_y=True)
    say(f"  oracle index built: n={ox.n}")
    vd, md = dev(vol), dev(mask)
    ix = nat.Index(vd, md, K, reduced_dim=D, n_curves=L, key_bits=b, window=W, curve=curve)
    info = ix.info
    assert info.n == ox.n and info.n_sub == ox.nsub and info.n_subsets == ox.S
    assert np.array_equal(host(ix.dictionary()), ox.dict)
    assert np.array_equal(host(ix.quantized()), ox.xq)
    assert np.float32(info.vmin) == ox.vmin and np.float32(info.qscale) == ox.qscale
    for s in range(ox.S):
        assert np.array_equal(ix.basis(s), ox.bases[s]), f"basis of subset {s}"
        lo, span = ix.params(s)
        assert np.array_equal(lo, ox.lo[s]) and span == ox.span[s], f"grid of subset {s}"
        assert np.array_equal(host(ix.projection(s)), ox.y[s]), f"projection of subset {s}"
        for j in range(L):
            k, i = ix.export(s, j)
            assert np.array_equal(host(k).view(np.uint64), ox.keys[s, j]), f"keys ({s},{j})"
            assert np.array_equal(host(i), ox.ids[s, j]), f"ids ({s},{j})"
    say(f"  {ox.S} bases, grids, projections and {ox.S * L} sorted curves equal")

    # the oracle's own front and targets; the GPU's front must equal it
    f = oracle.front(mask)
    assert np.array_equal(host(nat.fill_front(md)), f)
    rng = np.random.default_rng(22)
    sel = np.sort(rng.choice(f.size, 512, replace=False))
    t, m = oracle.extract(vol, mask, K, f[sel])
    _compare_queries(ix, ox, vol, t[:256], m[:256], "config2")

    bs, cs = (host(a) for a in ix.query(dev(t), dev(m), "fp32"))
    ob, oc = _brute_parallel(vol, mask.shape, K, ox.dict, t, m)
    assert np.array_equal(ob, bs)
    assert np.array_equal(oc.view(np.uint32), cs.view(np.uint32))
    say("  float32 scan equals the oracle's full scan on 512 queries")
    ix.close()


def _verify_subset_curves(ix, ox, s, L, b, curve, full_projection):
    """Verify subset s's grid and every sorted curve on the GPU against the
    oracle (see the module docstring) and attach the curves to ox."""
    n, D = ox.n, ox.D
    inv = np.full(ox.mask.size, -1, dtype=np.int64)   # voxel id -> dictionary rank
    inv[ox.dict] = np.arange(n)
    parts = _pool_map(lambda r: oracle.project(ox.xq, ox.shape, ox.K, ox.dict[r], ox.elems[s],
                                               ox.bases[s]), _slices(n))
    y = np.concatenate(parts)
    del parts
    lo, span = oracle.key_params(y)
    glo, gspan = ix.params(s)
    assert np.array_equal(glo, lo) and gspan == span, f"grid of subset {s}"
    if full_projection:
        assert np.array_equal(host(ix.projection(s)), y), f"projection of subset {s}"
    for j in range(L):
        kparts = _pool_map(lambda r: oracle.keys(y[r], lo, span, b, j, L, oracle.CURVES[curve]),
                           _slices(n))
        ko = np.concatenate(kparts).reshape(n, -1)   # the oracle's key of dictionary rank r
        del kparts
        k_, i_ = ix.export(s, j)
        keys, ids = host(k_).view(np.uint64).reshape(n, -1), host(i_)
        del k_, i_
        assert _increasing(keys, ids), f"curve ({s},{j}) not sorted by (key, id)"
        assert ids.min() >= 0 and ids.max() < inv.size, f"curve ({s},{j}): id out of range"
        rank = inv[ids]
        assert rank.min() >= 0, f"curve ({s},{j}): an id outside the dictionary"
        seen = np.zeros(n, dtype=bool)
        seen[rank] = True
        assert seen.all(), f"curve ({s},{j}) is not a permutation of the dictionary"
        del seen
        assert np.array_equal(keys, ko[rank]), f"curve ({s},{j}): keys differ from the oracle's"
        del ko, rank
        ox.attach_curve(s, j, lo, span, keys, ids)
        say(f"  curve ({s},{j}) verified: every key equals the oracle's")
    del y


def _run(name, n_queries, n_brute, check_bf16, n_index_subsets, n_index_queries):
    nat = need_gpu()
    d = getattr(synth, name)()
    vol, mask, K = d["volume"], d["mask"], d["K"]
    D, L, b, curve, W = d["D"], d["n_curves"], d["key_bits"], d["curve"], d["window"]
    say(f"{name}: {mask.shape} K={K} D={D} L={L} b={b} {curve} W={W}")
    vd, md = dev(vol), dev(mask)
    ix = nat.Index(vd, md, K, reduced_dim=D, n_curves=L, key_bits=b, window=W, curve=curve)
    info = ix.info
    say(f"  built: n={info.n}")

    # the oracle's statistics and bases (no curves), in a thread pool
    ox = oracle.Index(vol, mask, K, D, L, key_bits=b, curve=curve, window=W, threads=THREADS,
                      build_curves=False)
    er = minimum_filter(mask, size=K, mode="constant", cval=0)
    dict_ids = np.flatnonzero(er).astype(np.int64)
    assert np.array_equal(ox.dict, dict_ids)
    assert info.n == ox.n
    assert np.array_equal(host(ix.dictionary()), dict_ids)
    say("  dictionary ok")
    assert np.float32(info.vmin) == ox.vmin and np.float32(info.qscale) == ox.qscale
    assert info.n_sub == ox.nsub
    for s in range(ox.S):
        assert np.array_equal(ix.basis(s), ox.bases[s]), f"basis of subset {s}"
    say(f"  {ox.S} bases ok")

    # seeded front sample; the index queries are those whose subset (by the
    # oracle's rule) is among the most chosen ones
    f = oracle.front(mask)
    rng = np.random.default_rng(123)
    sel = np.sort(rng.choice(f.size, 4096, replace=False))
    t_all, m_all = oracle.extract(vol, mask, K, f[sel])
    subs = np.array([oracle.choose_subset(ox.pix, mm) for mm in m_all])
    top = [s for s, _ in sorted(Counter(subs.tolist()).items(), key=lambda x: (-x[1], x[0]))]
    top = sorted(top[:n_index_subsets])
    qi = np.flatnonzero(np.isin(subs, top))[:n_index_queries]
    assert qi.size == n_index_queries, f"only {qi.size} sampled queries in subsets {top}"
    for k, s in enumerate(top):
        _verify_subset_curves(ix, ox, s, L, b, curve, full_projection=(k == 0))
    bx_i, cx_i = _compare_queries(ix, ox, vol, t_all[qi], m_all[qi], name)
    ox.drop_curves()

    # the float32 scan and the index on a seeded sample
    t, m = t_all[:n_queries], m_all[:n_queries]
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
    _run("config3", n_queries=256, n_brute=32, check_bf16=True, n_index_subsets=2,
         n_index_queries=128)


def test_scale_phantom_512cube():
    _run("config4", n_queries=64, n_brute=32, check_bf16=False, n_index_subsets=1,
         n_index_queries=64)
