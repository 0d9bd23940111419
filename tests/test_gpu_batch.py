"""Batches of 2D images of uneven size and channel count, answered by one
persistent float32-scan launch captured in a HIP graph: every answer equals
the single-image float32 scan (and the oracle's full scan on a sample), on
every replay, after a layout change and with every tile-shape set."""
import numpy as np
import pytest
import torch

import oracle
from paper_1712_06326_amd import synth

from gpu_util import dev, host, need_gpu, say

pytestmark = pytest.mark.gpu


def _images(seed, count, lo, hi):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        h, w = (int(x) for x in rng.integers(lo, hi + 1, 2))
        c = int(rng.integers(1, 4))
        out.append(synth.small_image(h, w, c, seed * 100 + i))
    return out


def _queries(nat, imgs, K, keep=None):
    ts, ms, counts, fronts = [], [], [], []
    for i, d in enumerate(imgs):
        vd, md = dev(d["volume"]), dev(d["mask"])
        f = host(nat.fill_front(md))
        if keep is not None:
            f = f[: keep[i]]
        t, m = nat.extract_targets(vd, md, K, dev(f))
        ts.append(t.reshape(-1))
        ms.append(m)
        counts.append(f.size)
        fronts.append(f)
    return torch.cat(ts).contiguous(), torch.cat(ms).contiguous(), counts, fronts


def _single(nat, imgs, K, t, m, counts):
    """Answers of the single-image float32 scan, image by image."""
    ids, costs = [], []
    toff, qoff = 0, 0
    for d, q in zip(imgs, counts):
        C = d["volume"].shape[-1]
        ix = nat.Index(dev(d["volume"]), dev(d["mask"]), K)
        tq = t[toff: toff + q * K * K * C].reshape(q, K * K, C).contiguous()
        bi, bc = ix.query(tq, m[qoff: qoff + q].contiguous(), "fp32")
        ids.append(host(bi))
        costs.append(host(bc))
        ix.close()
        toff += q * K * K * C
        qoff += q
    return np.concatenate(ids), np.concatenate(costs)


@pytest.mark.parametrize("K,seed", [(5, 1), (9, 2), (7, 3)])
def test_batch_equals_single_image_scan(K, seed):
    nat = need_gpu()
    imgs = _images(seed, 6, 30, 110)
    say(f"batch K={K}: " + ", ".join(f"{d['volume'].shape}" for d in imgs))
    vols = [dev(d["volume"]) for d in imgs]
    masks = [dev(d["mask"]) for d in imgs]
    b = nat.Batch(vols, masks, K)
    t, m, counts, fronts = _queries(nat, imgs, K)
    bi, bc = b.query(t, m, counts)
    si, sc = _single(nat, imgs, K, t, m, counts)
    assert np.array_equal(host(bi), si)
    assert np.array_equal(host(bc).view(np.uint32), sc.view(np.uint32))
    # the oracle's full scan on the first two targets of each image
    qoff = 0
    for d, q, f in zip(imgs, counts, fronts):
        k = min(2, q)
        to, mo = oracle.extract(d["volume"], d["mask"], K, f[:k])
        ob, oc = oracle.brute(d["volume"], d["mask"].shape, K, oracle.dictionary(d["mask"], K),
                              to, mo)
        assert np.array_equal(ob, host(bi)[qoff: qoff + k])
        assert np.array_equal(oc.view(np.uint32), host(bc)[qoff: qoff + k].view(np.uint32))
        qoff += q
    st = b.stats()
    say(f"  {sum(counts)} queries, {st['work_items']} work items")
    b.close()


def test_batch_graph_replays_and_layout_change():
    nat = need_gpu()
    K = 9
    imgs = _images(7, 5, 40, 120)
    b = nat.Batch([dev(d["volume"]) for d in imgs], [dev(d["mask"]) for d in imgs], K)
    t, m, counts, _ = _queries(nat, imgs, K)
    out = (torch.empty(sum(counts), dtype=torch.int64, device="cuda"),
           torch.empty(sum(counts), dtype=torch.float32, device="cuda"))
    si, sc = _single(nat, imgs, K, t, m, counts)
    scratch = torch.zeros(1 << 20, device="cuda")
    for rep in range(4):
        out[0].fill_(-7)
        out[1].fill_(-1.0)
        bi, bc = b.query(t, m, counts, out)
        scratch.add_(1.0)            # eager work between replays
        torch.cuda.synchronize()
        assert np.array_equal(host(bi), si), f"replay {rep}"
        assert np.array_equal(host(bc).view(np.uint32), sc.view(np.uint32)), f"replay {rep}"
    assert b.stats()["graph_replays"] == 4
    # fewer queries for two images (one with none): a new layout, recaptured
    keep = [c for c in counts]
    keep[0] = 0
    keep[2] = max(1, counts[2] // 3)
    t2, m2, c2, _ = _queries(nat, imgs, K, keep)
    bi, bc = b.query(t2, m2, c2)
    si2, sc2 = _single(nat, imgs, K, t2, m2, c2)
    assert np.array_equal(host(bi), si2)
    assert np.array_equal(host(bc).view(np.uint32), sc2.view(np.uint32))
    b.close()


def test_batch_autotune():
    nat = need_gpu()
    K = 9
    imgs = _images(11, 4, 60, 160)
    b = nat.Batch([dev(d["volume"]) for d in imgs], [dev(d["mask"]) for d in imgs], K)
    t, m, counts, _ = _queries(nat, imgs, K)
    out = (torch.empty(sum(counts), dtype=torch.int64, device="cuda"),
           torch.empty(sum(counts), dtype=torch.float32, device="cuda"))
    v = b.autotune(t, m, counts, out)
    assert 0 <= v <= 2 and b.stats()["shape"] == v
    si, sc = _single(nat, imgs, K, t, m, counts)
    bi, bc = b.query(t, m, counts, out)
    assert np.array_equal(host(bi), si)
    assert np.array_equal(host(bc).view(np.uint32), sc.view(np.uint32))
    say(f"  autotuned shape set {v}")
    b.close()
