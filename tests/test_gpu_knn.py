"""GPU parity of the exact k-NN query (Section II.D): the outside-in
traversal of the unshifted Morton curve must return exactly the oracle's k
nearest grid cells (ties by id) and the same answer over them, bit for bit,
for one- to three-word keys, leaf sizes mu from 1 (splits down to single
cells) to above n (one leaf), k from 1 to 80, 2D and 3D, and the L1 cost."""
import numpy as np
import pytest

import oracle
from paper_1712_06326_amd import synth

from gpu_util import dev, host, need_gpu, say

pytestmark = pytest.mark.gpu


def _check(vol, mask, K, D, L, b, k, mu, norm="l2", stride=1):
    nat = need_gpu()
    say(f"knn {mask.shape}x{vol.shape[-1]} K={K} D={D} L={L} b={b} k={k} mu={mu} {norm}")
    ox = oracle.Index(vol, mask, K, D, L, key_bits=b, curve="morton", window=8, norm=norm)
    ix = nat.Index(dev(vol), dev(mask), K, reduced_dim=D, n_curves=L, key_bits=b, window=8,
                   curve="morton", norm=norm)
    f = oracle.front(mask)[::stride]
    t, m = oracle.extract(vol, mask, K, f)
    bi, bc, cand, nc = (host(a) for a in ix.knn(dev(t), dev(m), k=k, mu=mu, candidates=True))
    bo, co, cando, nco = ox.knn_query(vol, t, m, k=k)
    assert np.array_equal(nc, nco)
    assert np.array_equal(cand, cando)
    assert np.array_equal(bi, bo)
    assert np.array_equal(bc.view(np.uint32), co.view(np.uint32))
    ix.close()
    return ox


@pytest.mark.parametrize("h,w,c,K,D,L,b,k,mu,seed", [
    (40, 44, 1, 5, 4, 2, 8, 16, 8, 1),       # one key word
    (48, 64, 3, 5, 6, 3, 12, 80, 256, 2),    # two words
    (50, 70, 3, 9, 8, 4, 21, 80, 256, 3),    # three words (the config-2 key)
    (50, 70, 3, 9, 8, 4, 21, 1, 1, 3),       # k = 1, single-entry leaves
    (45, 52, 1, 7, 6, 4, 10, 40, 1, 4),      # deep traversal
    (36, 40, 2, 5, 12, 2, 9, 24, 32, 5),     # D above 8 (wider box arrays)
])
def test_knn_small_images(h, w, c, K, D, L, b, k, mu, seed):
    d = synth.small_image(h, w, c, seed)
    _check(d["volume"], d["mask"], K, D, L, b, k, mu)


@pytest.mark.parametrize("n,c,K,D,L,b,k,mu,seed", [
    (16, 1, 5, 8, 4, 8, 80, 64, 2),
    (18, 1, 7, 10, 6, 8, 32, 16, 3),
])
def test_knn_small_volumes(n, c, K, D, L, b, k, mu, seed):
    d = synth.small_volume(n, seed, c=c)
    _check(d["volume"], d["mask"], K, D, L, b, k, mu)


def test_knn_one_leaf_and_k_covering_the_dictionary():
    d = synth.small_image(18, 17, 2, 12, frac=0.08, holes=1)
    ox = _check(d["volume"], d["mask"], 5, 4, 2, 6, 200, 10 ** 6)
    assert ox.n <= 200


def test_knn_l1():
    d = synth.small_image(48, 64, 3, 7)
    _check(d["volume"], d["mask"], 5, 6, 3, 12, 32, 16, norm="l1")


def test_knn_config1():
    d = synth.config1()
    _check(d["volume"], d["mask"], 9, 8, 4, 8, 80, 256, stride=1)


def test_knn_argument_errors():
    nat = need_gpu()
    d = synth.small_image(30, 32, 1, 2)
    vd, md = dev(d["volume"]), dev(d["mask"])
    t, m = oracle.extract(d["volume"], d["mask"], 5, oracle.front(d["mask"])[:4])
    ix = nat.Index(vd, md, 5, reduced_dim=4, n_curves=2, curve="hilbert")
    with pytest.raises(nat.SfcError, match="Morton"):
        ix.knn(dev(t), dev(m))
    ix.close()
    ix = nat.Index(vd, md, 5, reduced_dim=4, n_curves=2)
    for k, mu in ((0, 8), (257, 8), (8, 0)):
        with pytest.raises(nat.SfcError):
            ix.knn(dev(t), dev(m), k=k, mu=mu)
    ix.close()
    ix = nat.Index(vd, md, 5, reduced_dim=8, n_curves=1, key_bits=30)
    with pytest.raises(nat.SfcError, match="62"):
        ix.knn(dev(t), dev(m))
    ix.close()
    ix = nat.Index(vd, md, 5)
    with pytest.raises(nat.SfcError, match="SFC index"):
        ix.knn(dev(t), dev(m))
    ix.close()
