"""The allocation-free float32 scan (sfc_query_fp32_noalloc) against the
float32 scan of sfc_query and the oracle: bit-exact ids and cost bits on two
calls in a row (the second smaller, so stale contents of the fixed array
would show), with every device allocation of the library made to fail during
the call, and a clear error above the array's capacity."""
import numpy as np
import pytest
import torch

import oracle
from paper_1712_06326_amd import synth

from gpu_util import dev, host, need_gpu, say

pytestmark = pytest.mark.gpu


def _targets(nat, vd, md, K):
    f = nat.fill_front(md)
    return nat.extract_targets(vd, md, K, f)


def _noalloc(nat, ix, t, m):
    Q = m.shape[0]
    bi = torch.full((Q,), -7, dtype=torch.int64, device=t.device)
    bc = torch.full((Q,), -7.0, dtype=torch.float32, device=t.device)
    nat.debug_fail_alloc(1)   # the library's next device allocation would fail
    try:
        ix.query_noalloc(t, m, bi, bc)
        torch.cuda.synchronize()
    finally:
        nat.debug_fail_alloc(0)
    return host(bi), host(bc)


@pytest.mark.parametrize("case", ["rgb_k9", "gray_k7", "vol_k5"])
def test_noalloc_equals_fp32_scan_on_two_calls(case):
    nat = need_gpu()
    if case == "rgb_k9":
        d, K = synth.small_image(70, 300, 3, 31), 9
    elif case == "gray_k7":
        d, K = synth.small_image(90, 120, 1, 32, holes=5), 7
    else:
        d, K = synth.small_volume(24, 33), 5
    vol, mask = d["volume"], d["mask"]
    say(f"noalloc {case}: {mask.shape}x{vol.shape[-1]} K={K}")
    vd, md = dev(vol), dev(mask)
    t, m = _targets(nat, vd, md, K)
    ix = nat.Index(vd, md, K)
    Q = m.shape[0]
    dict_ids = oracle.dictionary(mask, K)
    for call, q in enumerate([Q, max(1, Q // 3 - 5)]):
        tq, mq = t[:q].contiguous(), m[:q].contiguous()
        ri, rc = (host(a) for a in ix.query(tq, mq, "fp32"))
        ni, nc = _noalloc(nat, ix, tq, mq)
        assert np.array_equal(ni, ri), f"call {call}: ids differ from sfc_query"
        assert np.array_equal(nc.view(np.uint32), rc.view(np.uint32)), f"call {call}: cost bits"
        oi, oc = oracle.brute(vol, mask.shape, K, dict_ids, host(tq), host(mq))
        assert np.array_equal(ni, oi) and np.array_equal(nc.view(np.uint32), oc.view(np.uint32))
        say(f"  call {call}: {q} queries equal sfc_query and the oracle")
    ix.close()


def test_noalloc_refuses_above_capacity():
    nat = need_gpu()
    d = synth.small_image(40, 60, 3, 34)
    vd, md = dev(d["volume"]), dev(d["mask"])
    t, m = _targets(nat, vd, md, 9)
    ix = nat.Index(vd, md, 9)
    cap = 16 << 20
    q_big = 1
    while ix.noalloc_bytes(q_big) <= cap:
        q_big *= 2
    assert ix.noalloc_bytes(q_big) > cap and ix.noalloc_bytes(q_big // 2) <= cap
    bi = torch.empty(1, dtype=torch.int64, device="cuda")
    bc = torch.empty(1, dtype=torch.float32, device="cuda")
    # refused on the host before any launch: the pointers are never read
    L = nat.lib()
    rc = L.sfc_query_fp32_noalloc(ix._h, nat._ptr(t), nat._ptr(m), q_big, nat._ptr(bi),
                                  nat._ptr(bc))
    assert rc == -1 and b"bytes of scratch" in L.sfc_last_error()
    # the handle still answers afterwards
    ri, rc_ = (host(a) for a in ix.query(t, m, "fp32"))
    ni, nc = _noalloc(nat, ix, t, m)
    assert np.array_equal(ni, ri) and np.array_equal(nc.view(np.uint32), rc_.view(np.uint32))
    ix.close()
