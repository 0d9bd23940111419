"""The oracle's thread-pool helpers give the serial oracle's results: a pooled
index build (covariance subsample in slices, subsets in threads), a pooled
full scan (dictionary slices merged by (cost, id)), and an index whose curves
are attached one by one. CPU only."""
import numpy as np
import pytest

from paper_1712_06326_amd import synth


def test_pooled_index_and_scan_equal_serial(orc):
    d = synth.small_image(50, 60, 3, 3)
    vol, mask = d["volume"], d["mask"]
    a = orc.Index(vol, mask, 7, 6, 3, key_bits=12, window=8)
    b = orc.Index(vol, mask, 7, 6, 3, key_bits=12, window=8, threads=4)
    assert all(np.array_equal(x, y) for x, y in zip(a.bases, b.bases))
    assert np.array_equal(a.keys, b.keys) and np.array_equal(a.ids, b.ids)
    f = orc.front(mask)
    t, m = orc.extract(vol, mask, 7, f)
    ra, rb = a.query(vol, t, m), b.query(vol, t, m)
    assert all(np.array_equal(x, y) for x, y in zip(ra, rb))
    bi, bc = orc.brute(vol, mask.shape, 7, a.dict, t, m)
    pi, pc = orc.brute_pooled(vol, mask.shape, 7, a.dict, t, m, threads=5)
    assert np.array_equal(bi, pi) and np.array_equal(bc.view(np.uint32), pc.view(np.uint32))


@pytest.mark.parametrize("nd,K", [(2, 3), (2, 9), (3, 5), (3, 7)])
def test_pooled_dictionary_equals_serial(orc, nd, K):
    d = synth.small_image(61, 47, 1, 4) if nd == 2 else synth.small_volume(26, 3)
    mask = d["mask"]
    for threads in (2, 3, 5):
        assert np.array_equal(orc.dictionary_pooled(mask, K, threads), orc.dictionary(mask, K))


def test_pooled_scan_keeps_the_lowest_id_on_ties(orc):
    vol = np.full((30, 31, 1), 0.25, np.float32)
    mask = np.ones((30, 31), np.uint8)
    mask[12:15, 12:15] = 0
    d = orc.dictionary(mask, 5)
    t, m = orc.extract(vol, mask, 5, orc.front(mask))
    bi, _ = orc.brute_pooled(vol, mask.shape, 5, d, t, m, threads=7)
    assert np.all(bi == d[0])


def test_attached_curves_answer_as_built_ones(orc):
    d = synth.small_volume(14, 2)
    vol, mask = d["volume"], d["mask"]
    a = orc.Index(vol, mask, 5, 5, 2, key_bits=8, window=8)
    c = orc.Index(vol, mask, 5, 5, 2, key_bits=8, window=8, threads=3, build_curves=False)
    f = orc.front(mask)
    t, m = orc.extract(vol, mask, 5, f)
    subs = sorted({orc.choose_subset(a.pix, mm) for mm in m})
    with pytest.raises(ValueError):
        c.query(vol, t, m)
    for s in subs:
        for j in range(2):
            c.attach_curve(s, j, a.lo[s], a.span[s], a.keys[s, j], a.ids[s, j])
    ra, rc = a.query(vol, t, m), c.query(vol, t, m)
    assert all(np.array_equal(x, y) for x, y in zip(ra, rc))
