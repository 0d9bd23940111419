"""The reduced-precision full scan (exact-integer bf16 MFMA filter, exact
rescoring, float32 fallback) returns exactly the float32 scan's answer."""
import numpy as np
import pytest

import oracle
from paper_1712_06326_amd import synth

from gpu_util import dev, host, need_gpu, say

pytestmark = pytest.mark.gpu


def _same_as_oracle(vol, mask, K, Q=None, seed=0):
    nat = need_gpu()
    vd, md = dev(vol), dev(mask)
    f = host(nat.fill_front(md))
    if Q is not None and Q < f.size:
        f = np.sort(np.random.default_rng(seed).choice(f, Q, replace=False))
    t, m = nat.extract_targets(vd, md, K, dev(f))
    ix = nat.Index(vd, md, K)
    bi, bc = ix.query(t, m, "bf16")
    fb = ix.fallbacks()
    p1, p2 = ix.filter_tiles()
    assert 0 <= p2 <= p1 and p1 > 0
    say(f"  filter tiles: pass 1 {p1}, pass 2 {p2}")
    si, sc = ix.query(t, m, "fp32")
    assert np.array_equal(host(bi), host(si))
    assert np.array_equal(host(bc).view(np.uint32), host(sc).view(np.uint32))
    to, mo = oracle.extract(vol, mask, K, f)
    boi, boc = oracle.brute(vol, mask.shape, K, oracle.dictionary(mask, K), to, mo)
    assert np.array_equal(host(bi), boi)
    return fb, f.size


@pytest.mark.parametrize("h,w,c,K,seed", [(40, 44, 1, 3, 1), (37, 300, 3, 5, 2),
                                          (61, 530, 2, 7, 3), (50, 170, 3, 9, 4),
                                          (45, 45, 3, 11, 6)])
def test_reduced_small_images(h, w, c, K, seed):
    say(f"bf16 2D {h}x{w}x{c} K={K}")
    d = synth.small_image(h, w, c, seed)
    fb, q = _same_as_oracle(d["volume"], d["mask"], K)
    say(f"  fallbacks {fb}/{q}")


@pytest.mark.parametrize("n,c,K,seed", [(17, 2, 5, 2), (20, 1, 7, 3)])
def test_reduced_small_volumes(n, c, K, seed):
    d = synth.small_volume(n, seed, c=c)
    _same_as_oracle(d["volume"], d["mask"], K)


def test_reduced_config1():
    d = synth.config1()
    fb, q = _same_as_oracle(d["volume"], d["mask"], 9)
    say(f"config1 fallbacks {fb}/{q}")


def test_reduced_config2_sampled():
    """1024^2 RGB, several query tiles with a ragged last one: the bf16 scan
    equals the float32 scan on 700 front targets, and the oracle's full scan
    on a few of them."""
    nat = need_gpu()
    d = synth.config2()
    vol, mask = d["volume"], d["mask"]
    vd, md = dev(vol), dev(mask)
    f = host(nat.fill_front(md))
    f = np.sort(np.random.default_rng(9).choice(f, 700, replace=False))
    t, m = nat.extract_targets(vd, md, 9, dev(f))
    ix = nat.Index(vd, md, 9)
    bi, bc = ix.query(t, m, "bf16")
    p1, p2 = ix.filter_tiles()
    say(f"config2 700 queries: fallbacks {ix.fallbacks()}, filter tiles {p1} -> {p2}")
    assert p2 < p1
    si, sc = ix.query(t, m, "fp32")
    assert np.array_equal(host(bi), host(si))
    assert np.array_equal(host(bc).view(np.uint32), host(sc).view(np.uint32))
    to, mo = oracle.extract(vol, mask, 9, f[:3])
    boi, boc = oracle.brute(vol, mask.shape, 9, oracle.dictionary(mask, 9), to, mo)
    assert np.array_equal(host(bi)[:3], boi)


def test_reduced_seeded_by_index():
    """On a handle with an SFC index the index answers seed the threshold
    (one GEMM pass): the bf16 scan still equals the float32 scan."""
    nat = need_gpu()
    for name, K, D, L, b, Q in (("config1", 9, 8, 4, 8, None), ("config2", 9, 8, 4, 21, 600)):
        d = getattr(synth, name)()
        vol, mask = d["volume"], d["mask"]
        vd, md = dev(vol), dev(mask)
        f = host(nat.fill_front(md))
        if Q is not None:
            f = np.sort(np.random.default_rng(4).choice(f, Q, replace=False))
        t, m = nat.extract_targets(vd, md, K, dev(f))
        ix = nat.Index(vd, md, K, reduced_dim=D, n_curves=L, key_bits=b)
        bi, bc = ix.query(t, m, "bf16")
        fb = ix.fallbacks()
        p1, p2 = ix.filter_tiles()
        assert p1 > 0 and p2 == 0
        si, sc = ix.query(t, m, "fp32")
        assert np.array_equal(host(bi), host(si))
        assert np.array_equal(host(bc).view(np.uint32), host(sc).view(np.uint32))
        say(f"{name}: seeded bf16 == fp32 on {f.size} queries, fallbacks {fb}")
    d = synth.small_volume(20, 3, c=1)
    vol, mask = d["volume"], d["mask"]
    vd, md = dev(vol), dev(mask)
    f = nat.fill_front(md)
    t, m = nat.extract_targets(vd, md, 7, f)
    ix = nat.Index(vd, md, 7, reduced_dim=6, n_curves=3)
    bi, bc = ix.query(t, m, "bf16")
    si, sc = ix.query(t, m, "fp32")
    assert np.array_equal(host(bi), host(si))
    assert np.array_equal(host(bc).view(np.uint32), host(sc).view(np.uint32))


def test_reduced_small_lists_overflow_to_the_fp32_scan():
    """Lists of 64..256 entries overflow for many queries, while other
    workgroups are still appending: every query whose list lost a candidate
    must take the float32 scan (also when the count stopped exactly at the
    capacity), so both the two-pass and the seeded filter still equal the
    float32 scan, on every repetition."""
    nat = need_gpu()
    d = synth.config2()
    vol, mask = d["volume"], d["mask"]
    vd, md = dev(vol), dev(mask)
    f = host(nat.fill_front(md))
    f = np.sort(np.random.default_rng(12).choice(f, 1000, replace=False))
    t, m = nat.extract_targets(vd, md, 9, dev(f))
    plain = nat.Index(vd, md, 9)
    seeded = nat.Index(vd, md, 9, reduced_dim=8, n_curves=4, key_bits=21)
    si, sc = (host(a) for a in plain.query(t, m, "fp32"))
    try:
        for cap in (64, 256):
            nat.debug_list_capacity(cap)
            for name, ix in (("two-pass", plain), ("seeded", seeded)):
                for rep in range(3):
                    bi, bc = (host(a) for a in ix.query(t, m, "bf16"))
                    fb = ix.fallbacks()
                    say(f"  cap {cap} {name} rep {rep}: fallbacks {fb}/{f.size}")
                    if cap == 64:
                        assert fb > 0
                    assert np.array_equal(bi, si)
                    assert np.array_equal(bc.view(np.uint32), sc.view(np.uint32))
    finally:
        nat.debug_list_capacity(0)


def test_reduced_constant_and_duplicates():
    """Exact duplicates everywhere (a constant image): every cost ties at 0
    and the set overflows; the fallback still returns the lowest id."""
    nat = need_gpu()
    vol = np.full((40, 300, 1), 0.5, np.float32)
    mask = np.ones((40, 300), np.uint8)
    mask[18:22, 140:150] = 0
    vol[mask == 0] = 0
    vd, md = dev(vol), dev(mask)
    f = nat.fill_front(md)
    t, m = nat.extract_targets(vd, md, 5, f)
    ix = nat.Index(vd, md, 5)
    bi, bc = ix.query(t, m, "bf16")
    d0 = host(ix.dictionary())[0]
    assert np.all(host(bi) == d0) and np.all(host(bc) == 0.0)
    assert ix.fallbacks() == f.numel()


def test_reduced_target_outside_range_falls_back():
    nat = need_gpu()
    d = synth.small_image(40, 60, 2, 3)
    vol, mask = d["volume"], d["mask"]
    vd, md = dev(vol), dev(mask)
    f = nat.fill_front(md)
    t, m = nat.extract_targets(vd, md, 5, f)
    t = t.clone()
    t[0, 0, 0] = 7.0   # outside the byte-code range of the volume
    m = m.clone()
    m[0, 0] = 1
    ix = nat.Index(vd, md, 5)
    bi, bc = ix.query(t, m, "bf16")
    assert ix.fallbacks() >= 1   # query 0's bound is not valid
    si, sc = ix.query(t, m, "fp32")
    assert np.array_equal(host(bi), host(si))
    assert np.array_equal(host(bc).view(np.uint32), host(sc).view(np.uint32))
