"""Exact emulation of an approximate e4m3 cross-term filter (per-patch
scales) and its rigorous error bound, on the CPU.

For each sampled front target it counts the dictionary patches whose lower
bound  T2 - 2 X~ - 2 eps + N  reaches the exact optimum (the most favourable
threshold a certificate could use): the set a certified answer would have
to rescore. X~ is the cross term with both operands rounded to e4m3
(round to nearest even; per-patch scale max|v|/448, per-query scale
max|m t|/448), eps bounds |X - X~| elementwise (relative error 2^-4, plus
the subnormal step, plus float32 accumulation).

    python tests/fp8_bound_emulation.py [config2|small] [targets]
"""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1712_06326_amd import synth  # noqa: E402

U = 2.0 ** -4          # e4m3: 3 stored mantissa bits, half-ulp relative error
SUB = 2.0 ** -10       # half the subnormal step 2^-9
E4M3_MAX = 448.0


def e4m3(x):
    """Nearest e4m3 value (ties to even) of |x| <= 448."""
    a = np.abs(x).astype(np.float64)
    e = np.maximum(np.floor(np.log2(np.maximum(a, 1e-300))), -6.0)
    step = np.exp2(e - 3.0)
    return np.sign(x) * np.minimum(np.round(a / step) * step, E4M3_MAX)


def listed_counts(vol, mask, K, n_targets, seed=0):
    """(counts of listed patches per target, dictionary size, median bound /
    cost ratio per target)."""
    C = vol.shape[-1]
    dic = oracle.dictionary(mask, K)
    f = oracle.front(mask)
    rng = np.random.default_rng(seed)
    sel = np.sort(rng.choice(f.size, min(n_targets, f.size), replace=False))
    t, m = oracle.extract(vol, mask, K, f[sel])
    H, W = mask.shape
    h = K // 2
    offs = np.array([(dy - h) * W + (dx - h) for dy in range(K) for dx in range(K)])
    flat = vol.reshape(-1, C)
    P = K * K * C
    B = np.empty((dic.size, P), np.float32)
    step = 100000
    for i in range(0, dic.size, step):
        ids = dic[i:i + step]
        B[i:i + ids.size] = flat[ids[:, None] + offs[None, :]].reshape(ids.size, P)
    s_c = np.abs(B).max(1) / E4M3_MAX
    s_c[s_c == 0] = 1.0
    Bq = np.empty_like(B)
    for i in range(0, dic.size, step):
        sc = s_c[i:i + step, None]
        Bq[i:i + step] = (e4m3(B[i:i + step] / sc) * sc).astype(np.float32)
    absB = np.abs(B).astype(np.float64)
    counts, ratios = [], []
    for q in range(len(sel)):
        mq = np.repeat(m[q].astype(np.float64), C)
        tq = t[q].reshape(-1).astype(np.float64)
        a = tq * mq
        amax = np.abs(a).max()
        sig = amax / E4M3_MAX if amax > 0 else 1.0
        aq = e4m3(a / sig) * sig
        cost = ((tq[None, :] - B) ** 2 * mq[None, :]).sum(1)
        tau = cost.min()
        T2 = (a * a).sum()
        N = ((B.astype(np.float64) ** 2) * mq[None, :]).sum(1)
        Xt = Bq.astype(np.float64) @ aq
        da = U * np.abs(a) + sig * SUB
        eps = absB @ da + (np.abs(aq)[None, :] * (U * absB + s_c[:, None] * SUB)).sum(1)
        eps += P * 2.0 ** -24 * (np.abs(Bq).astype(np.float64) @ np.abs(aq))
        lb = T2 - 2.0 * Xt - 2.0 * eps + N
        counts.append(int((lb <= tau).sum()))
        ratios.append(float(np.median(eps / np.maximum(cost, 1e-12))))
    return np.array(counts), dic.size, np.array(ratios)


def main():
    name = sys.argv[1] if len(sys.argv) > 1 else "config2"
    nq = int(sys.argv[2]) if len(sys.argv) > 2 else 16
    d = synth.config2() if name == "config2" else synth.small_image(160, 170, 3, 41)
    counts, n, ratios = listed_counts(d["volume"], d["mask"], 9, nq)
    for i, (c, r) in enumerate(zip(counts, ratios)):
        print(f"target {i}: {c} of {n} patches listed, median bound / cost {r:.3f}")
    for cap in (2048, 16384, 85000, 262144):
        print(f"certified with list capacity {cap}: {100 * np.mean(counts <= cap):.1f}%")


if __name__ == "__main__":
    main()
