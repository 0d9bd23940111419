"""Error paths under allocation failure: every device allocation of an index
build and of its queries is made to fail in turn; each call either succeeds
or reports SFC_ENOMEM with the injected message, and a build afterwards still
answers exactly as before (no state left behind)."""
import numpy as np
import pytest

import oracle
from paper_1712_06326_amd import synth

from gpu_util import dev, host, need_gpu, say

pytestmark = pytest.mark.gpu

SFC_ENOMEM = -2


def _run(nat, vd, md, td, mq):
    ix = nat.Index(vd, md, 7, reduced_dim=4, n_curves=2)
    try:
        out = [tuple(host(x) for x in ix.query(td, mq, mode)) for mode in ("index", "fp32", "bf16")]
        out.append(tuple(host(x) for x in ix.knn(td, mq, k=16)))
    finally:
        ix.close()
    return out


def test_every_allocation_failure_is_reported():
    nat = need_gpu()
    d = synth.small_image(60, 64, 3, 9)
    vol, mask = d["volume"], d["mask"]
    f = oracle.front(mask)
    t, m = oracle.extract(vol, mask, 7, f)
    vd, md, td, mq = dev(vol), dev(mask), dev(t), dev(m)
    ref = _run(nat, vd, md, td, mq)
    failed = 0
    for n in range(1, 80):
        say(f"allocation {n} fails")
        nat.debug_fail_alloc(n)
        try:
            got = _run(nat, vd, md, td, mq)
        except nat.SfcError as e:
            assert e.code == SFC_ENOMEM and "injected allocation failure" in str(e), str(e)
            failed += 1
        else:
            for a, b in zip(ref, got):
                assert np.array_equal(a[0], b[0]) and np.array_equal(a[1].view(np.uint32),
                                                                     b[1].view(np.uint32))
        finally:
            nat.debug_fail_alloc(0)
    assert failed >= 20, failed
    after = _run(nat, vd, md, td, mq)
    for a, b in zip(ref, after):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1].view(np.uint32), b[1].view(np.uint32))
