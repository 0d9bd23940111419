"""GPU fill loop vs the oracle's: identical per-iteration logs (target centre,
chosen source, cost bits) and identical final volume and mask."""
import numpy as np
import pytest

import oracle
from paper_1712_06326_amd import synth

from gpu_util import dev, host, need_gpu, say

pytestmark = pytest.mark.gpu


def _run(vol, mask, K, order, mode, D=6, L=3, b=12, W=16):
    nat = need_gpu()
    say(f"inpaint {mask.shape}x{vol.shape[-1]} K={K} {order} {mode}")
    oix = oracle.Index(vol, mask, K, D, L, key_bits=b, window=W) if mode == "index" else None
    ov, om, olog = oracle.inpaint(vol, mask, K, order=order,
                                  mode="index" if mode == "index" else "brute", index=oix)
    vd, md = dev(vol.copy()), dev(mask.copy())
    ix = None
    if mode == "index":
        ix = nat.Index(vd, md, K, reduced_dim=D, n_curves=L, key_bits=b, window=W)
    it, glog = nat.inpaint(vd, md, K, order=order, mode=mode, index=ix, log_cap=100000)
    assert it == olog["iters"]
    assert np.array_equal(glog["centre"], olog["centre"])
    assert np.array_equal(glog["source"], olog["source"])
    assert np.array_equal(glog["cost"].view(np.uint32), olog["cost"].view(np.uint32))
    assert np.array_equal(host(md), om) and np.array_equal(host(vd), ov)
    return it


@pytest.mark.parametrize("order,mode", [("criminisi", "fp32"), ("raster", "fp32"),
                                        ("criminisi", "index"), ("criminisi", "bf16")])
def test_inpaint_small_image(order, mode):
    d = synth.small_image(40, 46, 3, 31, holes=2, frac=0.06)
    _run(d["volume"], d["mask"], 5, order, mode)


def test_inpaint_small_volume():
    d = synth.small_volume(14, 32, frac=0.03)
    _run(d["volume"], d["mask"], 3, "criminisi", "fp32")


def test_inpaint_config1_criminisi():
    d = synth.config1()
    it = _run(d["volume"], d["mask"], 9, "criminisi", "fp32")
    say(f"config1: {it} iterations")


def test_inpaint_config1_index():
    d = synth.config1()
    _run(d["volume"], d["mask"], 9, "criminisi", "index", D=8, L=4, b=8, W=32)


@pytest.mark.parametrize("order,mode", [("criminisi", "fp32"), ("raster", "index"),
                                        ("criminisi", "index")])
def test_inpaint_many_rounds(order, mode):
    # enough unknown voxels that the loop replays its 16-iteration graph
    # (rounds of floor(unknown / K^2) iterations) as well as single ones
    d = synth.small_image(80, 96, 2, 33, holes=4, frac=0.1)
    assert int((d["mask"] == 0).sum()) // 25 >= 16
    it = _run(d["volume"], d["mask"], 5, order, mode, D=6, L=3, b=10, W=16)
    say(f"  {it} iterations")


def test_inpaint_volume_index():
    d = synth.small_volume(18, 34, frac=0.04)
    _run(d["volume"], d["mask"], 5, "criminisi", "index", D=6, L=3, b=8, W=16)


def test_inpaint_two_level_pick():
    """Above 16,384 blocks of 256 voxels the pick reduces the block bests in
    two levels (`loop_part2_kernel`): a 164 x 160 x 160 volume (4,198,400
    voxels) of seeded noise with two small holes far apart, so that the
    targets alternate between distant second-level blocks."""
    rng = np.random.default_rng(41)
    shape = (164, 160, 160)
    vol = rng.random(shape, dtype=np.float32)[..., None]
    mask = np.ones(shape, np.uint8)
    mask[20:23, 20:23, 20:23] = 0
    mask[140:142, 130:132, 150:152] = 0
    assert mask.size > 16384 * 256
    it = _run(vol, mask, 3, "criminisi", "fp32")
    say(f"  {it} iterations")
