"""Index queries of a handful of targets, the fill loop's case: up to 256
targets the prologue runs a workgroup per target, and up to 32 targets the
rescoring splits each target's windows into shares of 8 to 64 entries, one
workgroup each, merged by a 64-bit atomic minimum. Subsets,
coordinates and answers equal the oracle's for batch sizes on both sides of
both switch points, in the L2 and L1 norms, on images and volumes, with
2 to 128 shares per target and ragged last shares, and call after call on
one handle (each call starts its packed minima afresh)."""
import numpy as np
import pytest

import oracle
from paper_1712_06326_amd import synth

from gpu_util import dev, host, need_gpu, say

pytestmark = pytest.mark.gpu

CASES = [
    # kind, size, channels, K, D, L, key bits, curve, W, norm, seed
    ("image", (50, 70), 3, 9, 8, 4, 21, "morton", 512, "l2", 11),    # 2048 entries, 128 shares
    ("image", (60, 64), 1, 7, 6, 4, 10, "hilbert", 300, "l1", 12),   # 1200 = 18 * 64 + 48
    ("image", (48, 64), 3, 5, 6, 3, 12, "morton", 16, "l2", 13),     # 48 = 32 + 16
    ("volume", 18, 1, 7, 10, 6, 8, "hilbert", 32, "l2", 14),         # 192 = 24 * 8
    ("volume", 16, 2, 5, 8, 4, 8, "morton", 64, "l1", 15),           # 256 = 16 * 16
]


@pytest.mark.parametrize("kind,size,c,K,D,L,b,curve,W,norm,seed", CASES)
def test_small_batches_equal_the_oracle(kind, size, c, K, D, L, b, curve, W, norm, seed):
    nat = need_gpu()
    if kind == "image":
        d = synth.small_image(size[0], size[1], c, seed)
    else:
        d = synth.small_volume(size, seed, c=c)
    vol, mask = d["volume"], d["mask"]
    say(f"small batches {kind} {mask.shape}x{c} K={K} D={D} L={L} W={W} {curve} {norm}")
    ox = oracle.Index(vol, mask, K, D, L, key_bits=b, curve=curve, window=W, norm=norm)
    ix = nat.Index(dev(vol), dev(mask), K, reduced_dim=D, n_curves=L, key_bits=b, window=W,
                   curve=curve, norm=norm)
    f = oracle.front(mask)
    order = np.random.default_rng(seed).permutation(f.size)
    for Q in (1, 7, 32, 33, 1, 256, 257, 5):
        sel = np.resize(f[order], Q)   # targets repeat once the front runs out
        t, m = oracle.extract(vol, mask, K, sel)
        td, mdq = dev(t), dev(m)
        sub, y = ix.coords(td, mdq)
        so, yo = ox.query_point(t, m)
        assert np.array_equal(host(sub), so), f"subsets, Q={Q}"
        assert np.array_equal(host(y).view(np.uint64), yo.view(np.uint64)), f"coordinates, Q={Q}"
        bi, bc = ix.query(td, mdq, "index")
        bo, co = ox.query(vol, t, m)[:2]
        assert np.array_equal(host(bi), bo), f"best ids, Q={Q}"
        assert np.array_equal(host(bc).view(np.uint32), co.view(np.uint32)), f"best costs, Q={Q}"
