"""GPU parity of the L1 cost variant (Section III.K): the float32 full scan
and the index's rescoring under the masked L1 sum, against the oracle's L1
full scan and L1 index, bit-exact in ids and cost bits; a hand case where
the L1 and L2 answers differ; and the modes that reject L1."""
import numpy as np
import pytest

import oracle
from paper_1712_06326_amd import synth

from gpu_util import dev, host, need_gpu, say

pytestmark = pytest.mark.gpu


def _scan_case(vol, mask, K, Q=None, seed=0):
    nat = need_gpu()
    vd, md = dev(vol), dev(mask)
    f = oracle.front(mask)
    rng = np.random.default_rng(seed)
    cen = f if Q is None or Q >= f.size else np.sort(rng.choice(f, Q, replace=False))
    t, m = oracle.extract(vol, mask, K, cen)
    ix = nat.Index(vd, md, K, norm="l1")
    do = host(ix.dictionary())
    bi, bc = (host(a) for a in ix.query(dev(t), dev(m), "fp32"))
    boi, boc = oracle.brute(vol, mask.shape, K, do, t, m, norm="l1")
    assert np.array_equal(bi, boi)
    assert np.array_equal(bc.view(np.uint32), boc.view(np.uint32))
    u = 2.0 ** -24
    for q in range(0, len(cen), max(1, len(cen) // 16)):
        e = oracle.cost64(vol, mask.shape, K, bi[q], t[q], m[q], norm="l1")
        k = int(m[q].sum()) * vol.shape[-1]
        assert abs(float(bc[q]) - e) <= (k + 1) * u * e or (e == 0 and bc[q] == 0)
    ix.close()


@pytest.mark.parametrize("h,w,c,K,seed", [
    (40, 44, 1, 5, 1), (37, 301, 3, 9, 2), (45, 70, 1, 9, 3), (33, 50, 3, 7, 4),
    (30, 41, 2, 3, 5), (48, 90, 3, 11, 6), (52, 60, 1, 13, 7),
])
def test_l1_scan_small_images(h, w, c, K, seed):
    d = synth.small_image(h, w, c, seed)
    say(f"L1 scan {h}x{w}x{c} K={K}")
    _scan_case(d["volume"], d["mask"], K)


@pytest.mark.parametrize("n,c,K,seed", [(14, 1, 3, 1), (17, 2, 5, 2), (20, 1, 7, 3),
                                        (18, 1, 5, 4)])
def test_l1_scan_small_volumes(n, c, K, seed):
    d = synth.small_volume(n, seed, c=c)
    say(f"L1 scan {n}^3x{c} K={K}")
    _scan_case(d["volume"], d["mask"], K)


def test_l1_and_l2_answers_differ_on_hand_case():
    nat = need_gpu()
    vol = np.zeros((3, 9, 1), np.float32)
    vol[1, :, 0] = [10, 1, 1, 1, 10, 0, 2.5, 0, 10]
    mask = np.ones((3, 9), np.uint8)
    t = np.zeros((1, 9, 1), np.float32)
    m = np.zeros((1, 9), np.uint8)
    m[0, 3:6] = 1
    vd, md = dev(vol), dev(mask)
    out = {}
    for norm in ("l2", "l1"):
        ix = nat.Index(vd, md, 3, norm=norm)
        bi, bc = ix.query(dev(t), dev(m), "fp32")
        out[norm] = (int(host(bi)[0]), float(host(bc)[0]))
        ix.close()
    assert out["l2"] == (11, 3.0) and out["l1"] == (15, 2.5)


@pytest.mark.parametrize("h,w,c,K,D,L,b,curve,W,seed", [
    (48, 64, 3, 5, 6, 3, 12, "morton", 16, 2),
    (50, 70, 3, 9, 8, 4, 21, "morton", 32, 3),
    (45, 52, 1, 7, 6, 4, 10, "hilbert", 16, 4),
])
def test_l1_index_small_images(h, w, c, K, D, L, b, curve, W, seed):
    nat = need_gpu()
    d = synth.small_image(h, w, c, seed)
    vol, mask = d["volume"], d["mask"]
    say(f"L1 index {h}x{w}x{c} K={K} D={D} L={L} b={b} {curve} W={W}")
    ox = oracle.Index(vol, mask, K, D, L, key_bits=b, curve=curve, window=W, norm="l1")
    ix = nat.Index(dev(vol), dev(mask), K, reduced_dim=D, n_curves=L, key_bits=b, window=W,
                   curve=curve, norm="l1")
    f = oracle.front(mask)
    t, m = oracle.extract(vol, mask, K, f)
    bi, bc = (host(a) for a in ix.query(dev(t), dev(m), "index"))
    bo, co, _, _, _ = ox.query(vol, t, m)
    assert np.array_equal(bi, bo)
    assert np.array_equal(bc.view(np.uint32), co.view(np.uint32))
    # the index never beats the L1 full scan
    bs, cs = (host(a) for a in ix.query(dev(t), dev(m), "fp32"))
    assert np.all(bc >= cs)
    ix.close()


def test_l1_rejected_where_unsupported():
    nat = need_gpu()
    d = synth.small_image(40, 44, 1, 9)
    vol, mask = d["volume"], d["mask"]
    vd, md = dev(vol), dev(mask)
    f = oracle.front(mask)[:8]
    t, m = oracle.extract(vol, mask, 5, f)
    ix = nat.Index(vd, md, 5, norm="l1")
    with pytest.raises(nat.SfcError, match="L1"):
        ix.query(dev(t), dev(m), "bf16")
    with pytest.raises(nat.SfcError, match="L1"):
        ix.autotune(dev(t), dev(m))
    ix.close()
    with pytest.raises(nat.SfcError, match="L2"):
        nat.Batch([vd], [md], 5, norm="l1")
    with pytest.raises(nat.SfcError, match="L2"):
        nat.inpaint(vd.clone(), md.clone(), 5, norm="l1")
