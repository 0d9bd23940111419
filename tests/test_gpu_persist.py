"""Saved indices (sfc_index_save / sfc_index_load): a loaded handle holds the
same stages as the saved one and answers every query mode bit for bit the
same; files made for another geometry, K, volume or mask are refused, and so
are truncated ones."""
import os

import numpy as np
import pytest

import oracle
from paper_1712_06326_amd import synth

from gpu_util import dev, host, need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("h,w,c,K,D,L,b,curve,seed", [
    (50, 70, 3, 9, 8, 4, 21, "morton", 3),
    (45, 52, 1, 7, 6, 4, 10, "hilbert", 4),
])
def test_saved_index_answers_the_same(tmp_path, h, w, c, K, D, L, b, curve, seed):
    nat = need_gpu()
    d = synth.small_image(h, w, c, seed)
    vol, mask = d["volume"], d["mask"]
    vd, md = dev(vol), dev(mask)
    say(f"save/load {h}x{w}x{c} K={K} D={D} L={L} b={b} {curve}")
    ix = nat.Index(vd, md, K, reduced_dim=D, n_curves=L, key_bits=b, window=16, curve=curve)
    path = tmp_path / "index.sfc"
    ix.save(path)
    assert os.path.getsize(path) > 0
    iy = nat.Index.load(vd, md, K, path)
    a, z = ix.info, iy.info
    for f in ("n", "n_sub", "n_subsets", "reduced_dim", "n_curves", "key_bits", "key_words",
              "window", "curve"):
        assert getattr(a, f) == getattr(z, f), f
    for s in range(a.n_subsets):
        assert np.array_equal(ix.basis(s), iy.basis(s))
        (lo1, sp1), (lo2, sp2) = ix.params(s), iy.params(s)
        assert np.array_equal(lo1, lo2) and sp1 == sp2
        for j in range(L):
            k1, i1 = ix.export(s, j)
            k2, i2 = iy.export(s, j)
            assert np.array_equal(host(k1), host(k2)) and np.array_equal(host(i1), host(i2))
    f = oracle.front(mask)
    t, m = oracle.extract(vol, mask, K, f)
    td, mq = dev(t), dev(m)
    for mode in ("index", "fp32", "bf16"):
        b1, c1 = (host(x) for x in ix.query(td, mq, mode))
        b2, c2 = (host(x) for x in iy.query(td, mq, mode))
        assert np.array_equal(b1, b2) and np.array_equal(c1.view(np.uint32), c2.view(np.uint32)), mode
    if curve == "morton":
        b1, c1 = (host(x) for x in ix.knn(td, mq, k=32))
        b2, c2 = (host(x) for x in iy.knn(td, mq, k=32))
        assert np.array_equal(b1, b2) and np.array_equal(c1.view(np.uint32), c2.view(np.uint32))
    ix.close()
    iy.close()


def test_saved_index_refuses_other_inputs(tmp_path):
    nat = need_gpu()
    d = synth.small_image(40, 44, 1, 5)
    vol, mask = d["volume"], d["mask"]
    vd, md = dev(vol), dev(mask)
    ix = nat.Index(vd, md, 5, reduced_dim=4, n_curves=2)
    path = tmp_path / "index.sfc"
    ix.save(path)
    ix.close()
    with pytest.raises(nat.SfcError, match="geometry"):
        nat.Index.load(vd, md, 7, path)
    mask2 = mask.copy()
    mask2[20, 20] = 1 - mask2[20, 20]
    with pytest.raises(nat.SfcError, match="another volume or mask"):
        nat.Index.load(vd, dev(mask2), 5, path)
    # the same value range, two known voxels' values swapped
    known = np.flatnonzero(mask.ravel() == 1)
    flat = vol.reshape(-1).copy()
    i, j = known[0], known[np.argmax(np.abs(flat[known] - flat[known[0]]))]
    flat[i], flat[j] = flat[j], flat[i]
    vol2 = flat.reshape(vol.shape)
    with pytest.raises(nat.SfcError, match="another volume or mask"):
        nat.Index.load(dev(vol2), md, 5, path)
    raw = open(path, "rb").read()
    bad = tmp_path / "cut.sfc"
    open(bad, "wb").write(raw[: len(raw) // 2])
    with pytest.raises(nat.SfcError, match="truncated"):
        nat.Index.load(vd, md, 5, bad)
    with pytest.raises(nat.SfcError):
        nat.Index.load(vd, md, 5, tmp_path / "missing.sfc")
    dct = nat.Index(vd, md, 5)
    with pytest.raises(nat.SfcError, match="dictionary-only"):
        dct.save(tmp_path / "x.sfc")
    dct.close()
