"""Pins of the CPU oracle against facts fixed by the paper or by mathematics.

Every test here runs on the CPU. Each targets a mistake that could hide in the
oracle (a dropped term, a wrong sign or index, a transposed operand), checking
it against something other than the oracle itself: values printed in the paper
(tests/golden), closed forms, library routines on independent formulations
(numpy/scipy), or exhaustive enumeration on tiny inputs.
"""
import json
import os

import numpy as np
import pytest
from scipy import ndimage

from paper_1712_06326_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _img(h=40, w=44, c=1, seed=7, frac=0.1, holes=2):
    d = synth.small_image(h, w, c, seed, holes=holes, frac=frac)
    return d["volume"], d["mask"]


# ------------------------------------------------------------------ front / extract / dictionary
@pytest.mark.parametrize("nd", [2, 3])
def test_front_is_known_next_to_unknown(orc, nd):
    rng = np.random.default_rng(3)
    shape = (23, 19) if nd == 2 else (9, 11, 7)
    mask = (rng.random(shape) > 0.2).astype(np.uint8)
    cross = ndimage.generate_binary_structure(nd, 1)
    want = (mask == 1) & ndimage.binary_dilation(mask == 0, structure=cross, border_value=0)
    got = orc.front(mask)
    assert np.array_equal(got, np.flatnonzero(want.ravel()))


def test_extract_matches_padded_slices(orc):
    vol, mask = _img(c=3)
    K, h = 7, 3
    cen = np.array([0, 45, 300, vol.shape[0] * vol.shape[1] - 1], dtype=np.int64)
    t, m = orc.extract(vol, mask, K, cen)
    H, W = mask.shape
    vp = np.zeros((H + 2 * h, W + 2 * h, 3), np.float32)
    mp = np.zeros((H + 2 * h, W + 2 * h), np.uint8)
    vp[h:-h, h:-h] = vol
    mp[h:-h, h:-h] = mask
    for q, c in enumerate(cen):
        y, x = divmod(int(c), W)
        mm = mp[y:y + K, x:x + K]
        tt = vp[y:y + K, x:x + K] * mm[..., None]
        assert np.array_equal(m[q].reshape(K, K), mm)
        assert np.array_equal(t[q].reshape(K, K, 3), tt)


@pytest.mark.parametrize("nd,K", [(2, 5), (2, 9), (3, 3), (3, 5)])
def test_dictionary_is_interior_erosion(orc, nd, K):
    rng = np.random.default_rng(nd * 10 + K)
    shape = (31, 28) if nd == 2 else (12, 13, 11)
    mask = (rng.random(shape) > 0.03).astype(np.uint8)
    er = ndimage.binary_erosion(mask == 1, structure=np.ones((K,) * nd), border_value=0)
    assert np.array_equal(orc.dictionary(mask, K), np.flatnonzero(er.ravel()))


# ------------------------------------------------------------------ cost and full scan
def test_verbatim_copy_costs_zero_and_is_found(orc):
    vol, mask = _img(c=3, seed=11)
    K = 5
    d = orc.dictionary(mask, K)
    cen = d[[3, 50, 200, len(d) - 1]]
    t, m = orc.extract(vol, mask, K, cen)
    bi, bc = orc.brute(vol, mask.shape, K, d, t, m)
    assert np.all(bc == 0.0)
    for q, c in enumerate(cen):
        # found id is the lowest id whose patch equals the target exactly
        assert bi[q] <= c
        t2, _ = orc.extract(vol, mask, K, [bi[q]])
        assert np.array_equal(t2[0], t[q])


def test_constant_image_returns_lowest_id(orc):
    vol = np.full((20, 21, 2), 0.25, np.float32)
    mask = np.ones((20, 21), np.uint8)
    mask[8:11, 9:12] = 0
    vol[mask == 0] = 0
    K = 3
    d = orc.dictionary(mask, K)
    f = orc.front(mask)
    t, m = orc.extract(vol, mask, K, f)
    bi, bc = orc.brute(vol, mask.shape, K, d, t, m)
    assert np.all(bc == 0.0) and np.all(bi == d[0])


def test_one_known_pixel_is_nearest_value(orc):
    vol, mask = _img(seed=5)
    K = 5
    d = orc.dictionary(mask, K)
    t = np.zeros((1, K * K, 1), np.float32)
    m = np.zeros((1, K * K), np.uint8)
    rho = 7  # offset (1, 2) -> (-1, 0)
    m[0, rho] = 1
    t[0, rho, 0] = np.float32(0.4321)
    bi, bc = orc.brute(vol, mask.shape, K, d, t, m)
    W = mask.shape[1]
    vals = vol.reshape(-1)[d - W]
    diff = (np.float32(0.4321) - vals).astype(np.float32)
    sq = (diff * diff).astype(np.float32)
    k = int(np.argmin(sq))  # first minimum = lowest id
    assert bi[0] == d[k] and bc[0] == sq[k]


def test_all_unknown_mask_costs_zero_lowest_id(orc):
    vol, mask = _img(seed=6)
    d = orc.dictionary(mask, 3)
    t = np.zeros((1, 9, 1), np.float32)
    m = np.zeros((1, 9), np.uint8)
    bi, bc = orc.brute(vol, mask.shape, 3, d, t, m)
    assert bi[0] == d[0] and bc[0] == 0.0


def test_cost_float32_vs_float64_and_numpy_bruteforce(orc):
    vol, mask = _img(h=36, w=30, c=3, seed=9)
    K = 5
    d = orc.dictionary(mask, K)
    f = orc.front(mask)[::7]
    t, m = orc.extract(vol, mask, K, f)
    bi, bc = orc.brute(vol, mask.shape, K, d, t, m)
    H, W = mask.shape
    off = (np.arange(K * K) // K - 2) * W + (np.arange(K * K) % K - 2)
    V = vol.reshape(-1, 3).astype(np.float64)
    for q in range(len(f)):
        patches = V[d[:, None] + off[None, :]]  # [n, K*K, 3]
        diff = (t[q].astype(np.float64)[None] - patches) * m[q][None, :, None]
        c64 = (diff ** 2).sum(axis=(1, 2))
        k = int(np.argmin(c64))
        gap = np.sort(c64)[1] - c64.min()
        # exact agreement unless the float64 runner-up is within rounding
        if gap > 1e-5 * max(c64.min(), 1e-30):
            assert bi[q] == d[k]
        e = orc.cost64(vol, mask.shape, K, bi[q], t[q], m[q])
        assert abs(float(bc[q]) - e) <= 1e-5 * max(e, 1e-30) or (bc[q] == 0 and e == 0)


# ------------------------------------------------------------------ L1 cost (Section III.K)
def test_l1_verbatim_copy_costs_zero_and_is_found(orc):
    vol, mask = _img(c=3, seed=11)
    K = 5
    d = orc.dictionary(mask, K)
    cen = d[[3, 50, 200, len(d) - 1]]
    t, m = orc.extract(vol, mask, K, cen)
    bi, bc = orc.brute(vol, mask.shape, K, d, t, m, norm="l1")
    assert np.all(bc == 0.0)
    for q, c in enumerate(cen):
        assert bi[q] <= c
        t2, _ = orc.extract(vol, mask, K, [bi[q]])
        assert np.array_equal(t2[0], t[q])


def test_l1_one_known_pixel_is_nearest_value(orc):
    vol, mask = _img(seed=5)
    K = 5
    d = orc.dictionary(mask, K)
    t = np.zeros((1, K * K, 1), np.float32)
    m = np.zeros((1, K * K), np.uint8)
    m[0, 7] = 1
    t[0, 7, 0] = np.float32(0.4321)
    bi, bc = orc.brute(vol, mask.shape, K, d, t, m, norm="l1")
    W = mask.shape[1]
    ad = np.abs((np.float32(0.4321) - vol.reshape(-1)[d - W]).astype(np.float32))
    k = int(np.argmin(ad))
    assert bi[0] == d[k] and bc[0] == ad[k]


def test_l1_and_l2_choose_different_patches(orc):
    # middle row known, target 0: candidate centre (1, 2) reads (1, 1, 1),
    # L1 = 3, L2 = 3; centre (1, 6) reads (0, 2.5, 0), L1 = 2.5, L2 = 6.25;
    # every other candidate meets a 10
    vol = np.zeros((3, 9, 1), np.float32)
    vol[1, :, 0] = [10, 1, 1, 1, 10, 0, 2.5, 0, 10]
    mask = np.ones((3, 9), np.uint8)
    K = 3
    d = orc.dictionary(mask, K)
    assert np.array_equal(d, 9 + np.arange(1, 8))
    t = np.zeros((1, 9, 1), np.float32)
    m = np.zeros((1, 9), np.uint8)
    m[0, 3:6] = 1
    b2, c2 = orc.brute(vol, mask.shape, K, d, t, m, norm="l2")
    b1, c1 = orc.brute(vol, mask.shape, K, d, t, m, norm="l1")
    assert (b2[0], c2[0]) == (11, 3.0)
    assert (b1[0], c1[0]) == (15, 2.5)
    assert orc.cost(vol, mask.shape, K, 15, t[0], m[0], norm="l2") == 6.25
    assert orc.cost(vol, mask.shape, K, 11, t[0], m[0], norm="l1") == 3.0


def test_l1_float32_vs_float64_and_numpy_bruteforce(orc):
    vol, mask = _img(h=36, w=30, c=3, seed=9)
    K = 5
    d = orc.dictionary(mask, K)
    f = orc.front(mask)[::7]
    t, m = orc.extract(vol, mask, K, f)
    bi, bc = orc.brute(vol, mask.shape, K, d, t, m, norm="l1")
    W = mask.shape[1]
    off = (np.arange(K * K) // K - 2) * W + (np.arange(K * K) % K - 2)
    V = vol.reshape(-1, 3).astype(np.float64)
    u = 2.0 ** -24
    for q in range(len(f)):
        patches = V[d[:, None] + off[None, :]]
        c64 = (np.abs(t[q].astype(np.float64)[None] - patches) * m[q][None, :, None]).sum(axis=(1, 2))
        k_terms = int(m[q].sum()) * 3
        tol = (k_terms + 1) * u   # k rounded differences and k - 1 rounded additions
        k = int(np.argmin(c64))
        gap = np.sort(c64)[1] - c64.min()
        if gap > 2 * tol * max(c64.min(), 1e-30):
            assert bi[q] == d[k]
        e = orc.cost64(vol, mask.shape, K, bi[q], t[q], m[q], norm="l1")
        assert abs(float(bc[q]) - e) <= tol * e or (bc[q] == 0 and e == 0)


def test_l1_index_equals_bruteforce_when_windows_cover_all(orc):
    vol, mask = _img(h=18, w=17, c=2, seed=12, frac=0.08, holes=1)
    K = 5
    ix = orc.Index(vol, mask, K, D=4, L=2, key_bits=6, window=256, norm="l1")
    assert ix.n <= 256
    f = orc.front(mask)
    t, m = orc.extract(vol, mask, K, f)
    bi, bc, _, nc, _ = ix.query(vol, t, m)
    b2, c2 = orc.brute(vol, mask.shape, K, ix.dict, t, m, norm="l1")
    assert np.array_equal(bi, b2) and np.array_equal(bc, c2)
    assert np.all(nc == ix.n)


# ------------------------------------------------------------------ quantisation
def test_quantize_hand_cases(orc):
    vol = np.array([[0.0, 1.0], [2.0, 0.5], [255.0 / 510.0 * 2.0, 9.0]], np.float32)[..., None]
    mask = np.array([[1, 1], [1, 1], [1, 0]], np.uint8)
    xq, vmin, s = orc.quantize(vol, mask)
    assert vmin == np.float32(0.0) and s == np.float32(255.0) / np.float32(2.0)
    assert xq[0, 0, 0] == 0 and xq[1, 0, 0] == 255       # vmin -> 0, vmax -> 255
    assert xq[0, 1, 0] == 128                            # 127.5 rounds to even 128
    assert xq[1, 1, 0] == 64                             # 0.5 * 127.5 = 63.75 -> 64
    assert xq[2, 1, 0] == 255                            # unknown voxel clamps
    flat = np.full((4, 4, 1), 3.0, np.float32)
    xq2, _, s2 = orc.quantize(flat, np.ones((4, 4), np.uint8))
    assert s2 == 0.0 and np.all(xq2 == 0)


# ------------------------------------------------------------------ pixel subsets
def test_subset_sizes_and_anchor_membership(orc):
    for nd, K, sizes in [(2, 9, {50}), (3, 7, {207, 208, 213}), (3, 5, {76, 78, 83})]:
        subs = orc.subsets(nd, K)
        assert len(subs) == 3 ** nd - 1
        assert set(p.size for p in subs) == sizes
        need = -(-6 * K ** nd // 10)
        for p in subs:
            assert p.size >= need and np.all(np.diff(p) > 0)


@pytest.mark.parametrize("nd,K", [(2, 9), (2, 7), (3, 5)])
def test_subsets_invariant_under_patch_symmetries(orc, nd, K):
    """Fig. 2: the four edge-midpoint subsets are rotations of each other, as
    are the four corner subsets; the whole family is invariant under the
    symmetry group of the square (cube)."""
    subs = orc.subsets(nd, K)
    boxes = []
    for p in subs:
        b = np.zeros(K ** nd, bool)
        b[p] = True
        boxes.append(b.reshape((K,) * nd))
    key = {b.tobytes() for b in boxes}
    axes = [(0, 1)] if nd == 2 else [(0, 1), (1, 2), (0, 2)]
    for b in boxes:
        for ax in axes:
            assert np.rot90(b, 1, axes=ax).tobytes() in key
        assert np.flip(b, 0).tobytes() in key


# ------------------------------------------------------------------ PCA
def _patches(xq, shape, K, ids):
    nd = len(shape)
    h = (K - 1) // 2
    strides = np.cumprod((1,) + tuple(shape[::-1]))[:-1][::-1]
    offs = np.zeros(K ** nd, np.int64)
    for rho in range(K ** nd):
        r = rho
        o = 0
        for i in range(nd - 1, -1, -1):
            o += ((r % K) - h) * strides[i]
            r //= K
        offs[rho] = o
    C = xq.shape[-1]
    X = xq.reshape(-1, C)[ids[:, None] + offs[None, :]]
    return X.reshape(len(ids), -1).astype(np.int64)


def test_cov_sums_match_numpy_int64(orc):
    vol, mask = _img(h=30, w=33, c=2, seed=4)
    K = 5
    xq, _, _ = orc.quantize(vol, mask)
    d = orc.dictionary(mask, K)
    s, ss, ns = orc.cov_sums(xq, mask.shape, K, d)
    X = _patches(xq, mask.shape, K, d)
    assert ns == len(d)
    assert np.array_equal(s, X.sum(0)) and np.array_equal(ss, X.T @ X)
    el = orc.subset_elems(orc.subsets(2, K)[3], 2)
    A = orc.cov_matrix(s, ss, ns, el)
    Ai = ns * (X[:, el].T @ X[:, el]) - np.outer(X[:, el].sum(0), X[:, el].sum(0))
    assert np.array_equal(A, Ai.astype(np.float64))


def test_cov_subsample_stride(orc):
    # n > 2^20 would need a large input; check the stride rule on the ids
    d = np.arange(3 * (1 << 20) + 5, dtype=np.int64)
    st = -(-d.size // (1 << 20))
    assert st == 4 and len(range(0, d.size, st)) == -(-d.size // st)


@pytest.mark.parametrize("m", [7, 12, 50])
def test_jacobi_matches_eigh(orc, m):
    rng = np.random.default_rng(m)
    X = rng.integers(0, 256, size=(400, m)).astype(np.float64)
    X[:, 1] = X[:, 0]  # a repeated column: a zero eigenvalue
    A = 400 * X.T @ X - np.outer(X.sum(0), X.sum(0))
    Ad, V, sweeps = orc.jacobi(A)
    lam = np.diag(Ad)
    ref = np.linalg.eigh(A)
    assert sweeps < 60
    assert np.allclose(np.sort(lam), ref[0], rtol=1e-11, atol=1e-9 * ref[0].max())
    assert np.abs(V.T @ V - np.eye(m)).max() < 1e-12
    assert np.abs(A @ V - V * lam).max() < 1e-9 * ref[0].max()


def test_basis_orders_signs_and_scales(orc):
    rng = np.random.default_rng(2)
    m, D = 20, 6
    X = rng.integers(0, 256, size=(300, m)).astype(np.float64) @ rng.normal(size=(m, m))
    A = X.T @ X
    Ad, V, _ = orc.jacobi(A)
    w, order = orc.basis_from(Ad, V, D)
    lam, U = np.linalg.eigh(A)
    U = U[:, ::-1][:, :D]
    U = U * np.sign(U[np.abs(U).argmax(0), np.arange(D)])
    g = np.abs(U).max()
    assert np.abs(w).max() == 127
    assert np.abs(w.astype(np.float64) - U * 127 / g).max() <= 0.5 + 1e-6
    assert np.all(np.diff(np.diag(Ad)[order]) <= 0)


def _eigh_basis(A, D):
    """rint(127 U / g) from numpy's eigh: U the D leading eigenvectors
    (eigenvalue descending), each signed positive at its largest-magnitude
    entry, g the largest magnitude over them; also the distance of every
    scaled entry from a rounding tie."""
    lam, U = np.linalg.eigh(A)
    U = U[:, ::-1][:, :D]
    U = U * np.sign(U[np.abs(U).argmax(0), np.arange(D)])
    z = U * 127 / np.abs(U).max()
    tie = np.abs(np.abs(z - np.floor(z)) - 0.5)
    return np.rint(z), tie, lam[::-1]


def _real_cov(orc, nd, K, C, seed, subset):
    if nd == 2:
        d = synth.small_image(48, 52, C, seed, holes=2, frac=0.08)
    else:
        d = synth.small_volume(22, seed)
    vol, mask = d["volume"], d["mask"]
    xq, _, _ = orc.quantize(vol, mask)
    dd = orc.dictionary(mask, K)
    s, ss, ns = orc.cov_sums(xq, mask.shape, K, dd)
    el = orc.subset_elems(orc.subsets(nd, K)[subset], vol.shape[-1])
    return orc.cov_matrix(s, ss, ns, el)


@pytest.mark.parametrize("case", ["rand7", "rand12", "rand50", "mixed20",
                                  "img2d_k9_c3_s0", "img2d_k9_c3_s5", "img2d_k7_c1_s2",
                                  "vol3d_k5_s0", "vol3d_k5_s13", "vol3d_k7_s4"])
def test_basis_equals_rounded_eigh(orc, case):
    # The int8 basis depends only on the eigenvectors, not on the Jacobi
    # solver's rounding order (its round-robin pairing, its mirroring of the
    # upper triangle): every entry equals rint(127 U / g) computed from
    # numpy's eigh, except entries within 1e-9 of a rounding tie.
    D = 8
    if case.startswith("rand"):
        m = int(case[4:])
        rng = np.random.default_rng(m)
        X = rng.integers(0, 256, size=(400, m)).astype(np.float64)
        X[:, 1] = X[:, 0]
        A = 400 * X.T @ X - np.outer(X.sum(0), X.sum(0))
        D = min(D, m - 2)
    elif case == "mixed20":
        rng = np.random.default_rng(2)
        X = rng.integers(0, 256, size=(300, 20)).astype(np.float64) @ rng.normal(size=(20, 20))
        A = X.T @ X
        D = 6
    elif case.startswith("img2d"):
        _, k, c, s = case.split("_")
        A = _real_cov(orc, 2, int(k[1:]), int(c[1:]), 3, int(s[1:]))
    else:
        _, k, s = case.split("_")
        A = _real_cov(orc, 3, int(k[1:]), 1, 4, int(s[1:]))
    Ad, V, _ = orc.jacobi(A)
    w, order = orc.basis_from(Ad, V, D)
    want, tie, lam = _eigh_basis(A, D)
    # the eigenvectors must be well defined: distinct leading eigenvalues
    gaps = np.abs(np.diff(lam[:D + 1]))
    assert gaps.min() > 1e-6 * lam[0]
    ok = tie > 1e-9
    assert ok.mean() > 0.99
    assert np.array_equal(w.astype(np.float64)[ok], want[ok])
    assert np.all(np.abs(w.astype(np.float64) - want) <= 1)


def test_projection_matches_numpy(orc):
    vol, mask = _img(h=26, w=29, c=3, seed=8)
    K = 5
    xq, _, _ = orc.quantize(vol, mask)
    d = orc.dictionary(mask, K)
    el = orc.subset_elems(orc.subsets(2, K)[0], 3)
    w = np.random.default_rng(1).integers(-127, 128, size=(el.size, 4)).astype(np.int8)
    y = orc.project(xq, mask.shape, K, d, el, w)
    X = _patches(xq, mask.shape, K, d)
    assert np.array_equal(y, X[:, el] @ w.astype(np.int64))


# ------------------------------------------------------------------ keys
def test_morton_matches_hand_table(orc):
    g = json.load(open(os.path.join(GOLD, "zorder_4x4.json")))
    for v0 in range(4):
        for v1 in range(4):
            assert int(orc.key_of([v0, v1], g["bits"], 0)[0]) == g["keys"][v0][v1]


def test_morton_one_dim_is_identity(orc):
    for b in (1, 5, 21, 31):
        for v in (0, 1, (1 << b) - 1, (1 << b) // 3):
            assert int(orc.key_of([v], b, 0)[0]) == v


def _msb_dim_less(a, b):
    """Z-order comparison as described in Section II.C: find the dimension
    holding the most significant differing bit (the first such dimension on
    equal bit levels) and compare only that dimension."""
    best, level = None, -1
    for d, (x, y) in enumerate(zip(a, b)):
        lv = (int(x) ^ int(y)).bit_length() - 1
        if lv > level:
            best, level = d, lv
    return best is not None and a[best] < b[best]


def _key_int(words):
    v = 0
    for w in words:
        v = (v << 64) | int(w)
    return v


@pytest.mark.parametrize("D,b", [(2, 3), (8, 8), (10, 8), (8, 21), (12, 21)])
def test_morton_key_order_equals_msb_comparator(orc, D, b):
    rng = np.random.default_rng(D * 100 + b)
    for _ in range(300):
        a = rng.integers(0, 1 << b, D)
        c = a.copy()
        k = rng.integers(0, D)
        c[k:] = rng.integers(0, 1 << b, D - k)  # share a prefix sometimes
        ka, kc = _key_int(orc.key_of(a, b, 0)), _key_int(orc.key_of(c, b, 0))
        assert (ka < kc) == _msb_dim_less(a, c)
        assert (ka == kc) == bool(np.all(a == c))
        assert ka < (1 << (D * b))


def test_fig3_box_interval(orc):
    g = json.load(open(os.path.join(GOLD, "fig3_box.json")))
    b = g["bits"]
    key = {(x, y): int(orc.key_of([x, y], b, 0)[0]) for x in range(8) for y in range(8)}
    mn, mx = tuple(g["box_min"]), tuple(g["box_max"])
    box = [(x, y) for x in range(mn[0], mx[0] + 1) for y in range(mn[1], mx[1] + 1)]
    assert all(key[mn] <= key[p] <= key[mx] for p in box)
    lower = [p for p in box if p[1] <= 3]
    upper = [p for p in box if p[1] >= 4]
    assert max(lower, key=key.get) == tuple(g["litmax"])
    assert min(upper, key=key.get) == tuple(g["bigmin"])
    gap = [p for p, k in key.items() if key[tuple(g["litmax"])] < k < key[tuple(g["bigmin"])]]
    assert gap and not any(p in box for p in gap)


@pytest.mark.parametrize("D,b", [(2, 1), (2, 2), (2, 4), (3, 2), (3, 4), (4, 2)])
def test_hilbert_bijective_and_adjacent(orc, D, b):
    pts = np.array(np.meshgrid(*[np.arange(1 << b)] * D, indexing="ij")).reshape(D, -1).T
    keys = np.array([_key_int(orc.key_of(p, b, 1)) for p in pts])
    assert np.array_equal(np.sort(keys), np.arange(1 << (D * b)))
    order = pts[np.argsort(keys)]
    assert np.all(order[0] == 0)
    steps = np.abs(np.diff(order, axis=0)).sum(1)
    assert np.all(steps == 1)


def test_hilbert_sampled_adjacency_high_dim(orc):
    D, b = 10, 2
    rng = np.random.default_rng(0)
    for _ in range(200):
        p = rng.integers(0, 1 << b, D)
        k = _key_int(orc.key_of(p, b, 1))
        # the successor along the curve is a unit step away
        nxt = None
        for d in range(D):
            for s in (-1, 1):
                q = p.copy()
                q[d] += s
                if 0 <= q[d] < (1 << b) and _key_int(orc.key_of(q, b, 1)) == k + 1:
                    nxt = q
        assert nxt is not None or k == (1 << (D * b)) - 1


def test_key_cells_and_shifts(orc):
    y = np.array([[0, 5], [10, -3], [4, 7]], np.int64)
    lo, span = orc.key_params(y)
    assert list(lo) == [0, -3] and span == 10
    b, L = 8, 3
    k0 = orc.keys(y, lo, span, b, 0, L, 0)
    R = 1 << (b - 1)
    # the minimum corner maps to the zero cell on the unshifted curve
    assert _key_int(orc.key_of([0, 0], b, 0)) == 0
    assert _key_int(k0[0]) == _key_int(orc.key_of([0, (8 * (R - 1)) // 10], b, 0))
    assert _key_int(k0[1]) == _key_int(orc.key_of([R - 1, 0], b, 0))
    # curve j adds floor(j*R/(D+1)) on every dim
    sh = (2 * R) // 3
    k2 = orc.keys(y, lo, span, b, 2, L, 0)
    assert _key_int(k2[1]) == _key_int(orc.key_of([R - 1 + sh, sh], b, 0))


def test_sort_is_sorted_permutation(orc):
    rng = np.random.default_rng(5)
    k = rng.integers(0, 4, size=(500, 2)).astype(np.uint64)
    ids = rng.permutation(500).astype(np.int64)
    ks, idss = orc.sort(k, ids)
    assert np.array_equal(np.sort(idss), np.sort(ids))
    tup = [(int(a), int(b), int(i)) for (a, b), i in zip(ks, idss)]
    assert tup == sorted(tup)
    ref = {int(i): (int(a), int(b)) for (a, b), i in zip(k, ids)}
    assert all(ref[int(i)] == (int(a), int(b)) for (a, b), i in zip(ks, idss))


# ------------------------------------------------------------------ index query
def test_index_equals_bruteforce_when_windows_cover_all(orc):
    vol, mask = _img(h=18, w=17, c=2, seed=12, frac=0.08, holes=1)
    K = 5
    ix = orc.Index(vol, mask, K, D=4, L=2, key_bits=6, window=256)
    assert ix.n <= 256
    f = orc.front(mask)
    t, m = orc.extract(vol, mask, K, f)
    bi, bc, cand, nc, _ = ix.query(vol, t, m)
    b2, c2 = orc.brute(vol, mask.shape, K, ix.dict, t, m)
    assert np.array_equal(bi, b2) and np.array_equal(bc, c2)
    assert np.all(nc == ix.n)


def test_index_finds_verbatim_copies_with_unique_keys(orc):
    vol, mask = _img(h=48, w=52, c=3, seed=13)
    K = 5
    ix = orc.Index(vol, mask, K, D=6, L=2, key_bits=12, window=8)
    sel = ix.dict[::37]
    t, m = orc.extract(vol, mask, K, sel)
    bi, bc, cand, nc, sub = ix.query(vol, t, m)
    hits = 0
    for q, c in enumerate(sel):
        s = sub[q]
        k = ix.keys[s, 0]
        pos = int(np.flatnonzero(ix.ids[s, 0] == c)[0])
        same = np.all(k == k[pos], axis=1).sum()
        if same == 1:
            hits += 1
            assert bc[q] == 0.0 and c in cand[q]
    assert hits > len(sel) // 2


# ------------------------------------------------------------------ exact k-NN query (Section II.D)
@pytest.mark.parametrize("D,b", [(2, 4), (5, 8), (8, 21), (10, 8), (16, 12)])
def test_morton_decode_inverts_the_interleave(orc, D, b):
    rng = np.random.default_rng(D * 100 + b)
    for _ in range(50):
        v = rng.integers(0, 1 << b, size=D, dtype=np.uint32)
        assert np.array_equal(orc.morton_decode(orc.key_of(v, b, 0), D, b), v)


def test_knn_equals_full_scan_when_k_covers_dictionary(orc):
    vol, mask = _img(h=18, w=17, c=2, seed=12, frac=0.08, holes=1)
    K = 5
    ix = orc.Index(vol, mask, K, D=4, L=2, key_bits=6, window=8)
    f = orc.front(mask)
    t, m = orc.extract(vol, mask, K, f)
    bi, bc, cand, nc = ix.knn_query(vol, t, m, k=ix.n + 5)
    b2, c2 = orc.brute(vol, mask.shape, K, ix.dict, t, m)
    assert np.array_equal(bi, b2) and np.array_equal(bc.view(np.uint32), c2.view(np.uint32))
    assert np.all(nc == ix.n) and np.all(cand[:, :ix.n] == ix.dict[None, :])


def test_knn_set_is_the_k_nearest_cells(orc):
    # cells recomputed in numpy from the projections (not from the keys),
    # squared distances, k smallest by (distance, id)
    vol, mask = _img(h=40, w=44, c=1, seed=3)
    K, D, L, b, k = 5, 4, 3, 10, 20
    ix = orc.Index(vol, mask, K, D=D, L=L, key_bits=b, window=8, keep_y=True)
    R = 1 << (b - 1)
    f = orc.front(mask)[::5]
    t, m = orc.extract(vol, mask, K, f)
    _, _, cand, nc = ix.knn_query(vol, t, m, k=k)
    sub, yq = ix.query_point(t, m)
    for q in range(len(f)):
        s = sub[q]
        lo, span = ix.lo[s], ix.span[s]
        cells = np.clip(np.floor_divide((ix.y[s] - lo) * (R - 1), span), 0, R - 1)
        uq = np.clip(np.floor(((yq[q] - lo) * (R - 1)) / span), 0, R - 1).astype(np.int64)
        dist = ((cells - uq[None, :]) ** 2).sum(axis=1)
        order = np.lexsort((ix.dict, dist))[:k]
        assert nc[q] == k
        assert np.array_equal(cand[q], np.sort(ix.dict[order]))


def test_knn_finds_verbatim_copies(orc):
    vol, mask = _img(h=36, w=40, c=3, seed=21)
    K = 5
    ix = orc.Index(vol, mask, K, D=6, L=2, key_bits=12, window=8)
    cen = ix.dict[[5, 77, 300, ix.n - 2]]
    t, m = orc.extract(vol, mask, K, cen)
    _, bc, _, _ = ix.knn_query(vol, t, m, k=16)
    assert np.all(bc == 0.0)


def test_knn_needs_a_morton_index(orc):
    vol, mask = _img(h=20, w=22, c=1, seed=2)
    ix = orc.Index(vol, mask, 3, D=2, L=2, key_bits=6, curve="hilbert")
    t, m = orc.extract(vol, mask, 3, orc.front(mask)[:2])
    with pytest.raises(ValueError):
        ix.knn_query(vol, t, m, k=4)


def test_knn_rejects_keys_whose_distances_could_overflow(orc):
    # D * (2^b)^2 must stay below 2^62: D=8, b=30 gives 2^63 and is refused;
    # D=4, b=30 gives exactly 2^62 and still ranks the dictionary exactly
    vol, mask = _img(h=20, w=22, c=1, seed=3)
    t, m = orc.extract(vol, mask, 5, orc.front(mask)[:3])
    ix = orc.Index(vol, mask, 5, D=8, L=1, key_bits=30)
    with pytest.raises(ValueError):
        ix.knn_query(vol, t, m, k=4)
    ix = orc.Index(vol, mask, 5, D=4, L=1, key_bits=30)
    bi, bc, _, nc = ix.knn_query(vol, t, m, k=ix.n + 5)
    b2, c2 = orc.brute(vol, mask.shape, 5, ix.dict, t, m)
    assert np.all(nc == ix.n)
    assert np.array_equal(bi, b2) and np.array_equal(bc.view(np.uint32), c2.view(np.uint32))


def test_query_coords_full_mask_exact_and_partial_least_squares(orc):
    import ctypes
    vol, mask = _img(h=40, w=40, c=1, seed=14)
    K = 5
    ix = orc.Index(vol, mask, K, D=5, L=2, key_bits=12, window=16, keep_y=True)
    L = orc.lib()
    L.orc_query_point.restype = ctypes.c_int
    L.orc_query_point.argtypes = [ctypes.POINTER(orc.OrcIndex), ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p]
    cen = ix.dict[[10, 100, 250]]
    t, m = orc.extract(vol, mask, K, cen)
    for q in range(len(cen)):
        yq = np.zeros(64)
        s = L.orc_query_point(ctypes.byref(ix.struct()), t[q].ctypes.data, m[q].ctypes.data,
                              yq.ctypes.data)
        assert s == 0  # full coverage everywhere: ties to the first subset
        i = int(np.flatnonzero(ix.dict == cen[q])[0])
        assert np.array_equal(yq[:5], ix.y[0][i].astype(np.float64))
        # hide a third of the pixels: the least-squares completion, solved
        # independently with numpy on the unridged problem, agrees closely
        mh = m[q].copy()
        mh[::3] = 0
        s = L.orc_query_point(ctypes.byref(ix.struct()), t[q].ctypes.data, mh.ctypes.data,
                              yq.ctypes.data)
        pix = ix.pix[s]
        W = ix.bases[s].astype(np.float64)
        kn = mh[pix].astype(bool)
        x = np.clip(np.rint((t[q][pix, 0] - ix.vmin) * ix.qscale), 0, 255)
        mu = ix.sum[pix] / ix.nsub
        a = np.linalg.lstsq(W[kn], x[kn] - mu[kn], rcond=None)[0]
        ref = W[kn].T @ x[kn] + W[~kn].T @ (mu[~kn] + W[~kn] @ a)
        assert np.allclose(yq[:5], ref, rtol=1e-4, atol=1.0)


def _mask_3d_k5(unknown):
    """A 5x5x5 target pixel mask with the pixels whose (i, j, k) satisfies
    unknown(i, j, k) set to 0 (rho = 25 i + 5 j + k)."""
    m = np.ones(125, np.uint8)
    for r in range(125):
        if unknown(r // 25, (r // 5) % 5, r % 5):
            m[r] = 0
    return m


def _fraction_rule(pix, m):
    """The reading of Fig. 1b: the subset with the largest known fraction,
    ties to the lower subset, in exact rationals."""
    from fractions import Fraction
    fr = [Fraction(int(m[p].sum()), p.size) for p in pix]
    return fr.index(max(fr)), fr


def test_subset_choice_is_largest_known_fraction_not_count(orc):
    # 3D, K = 5: anchors {0, 2, 4}^3 minus the centre in lexicographic order,
    # so subset 18 is anchored at (4, 0, 2) (an edge midpoint, 83 pixels) and
    # subset 21 at (4, 2, 2) (the face centre, 76 pixels). With the plane
    # i = 0 unknown, the face-centre subset opposite it is fully known (76 of
    # 76) while the edge subset keeps the most known pixels (79 of 83): the
    # largest known fraction picks 21, the largest known count would pick 18.
    pix = orc.subsets(3, 5)
    m = _mask_3d_k5(lambda i, j, k: i == 0)
    counts = [int(m[p].sum()) for p in pix]
    assert (pix[21].size, counts[21]) == (76, 76) and (pix[18].size, counts[18]) == (83, 79)
    assert int(np.argmax(counts)) == 18
    assert _fraction_rule(pix, m)[0] == 21
    assert orc.choose_subset(pix, m) == 21
    # the fraction-rule winner is unique here, so taking the smallest fraction
    # or the last subset would differ too
    assert orc.choose_subset(pix, 1 - m) != 21


def test_subset_choice_ties_go_to_the_lower_subset(orc):
    # The line (i, 2, 2), i = 0..4, through the centre unknown: eight edge
    # subsets (1, 3, 5, 7, 18, 20, 22, 24) each lose four of their 83 pixels
    # and tie at 79/83, the largest fraction (no subset is fully known); the
    # lowest of them, 1, is chosen (the highest would be 24).
    pix = orc.subsets(3, 5)
    m = _mask_3d_k5(lambda i, j, k: j == 2 and k == 2)
    best, fr = _fraction_rule(pix, m)
    from fractions import Fraction
    tied = [s for s, f in enumerate(fr) if f == max(fr)]
    assert tied == [1, 3, 5, 7, 18, 20, 22, 24] and max(fr) == Fraction(79, 83)
    assert orc.choose_subset(pix, m) == 1
    # a full mask ties every subset at 1: subset 0
    assert orc.choose_subset(pix, np.ones(125, np.uint8)) == 0


def test_subset_choice_seeded_masks_follow_the_fraction_rule(orc):
    # seeded partial masks in 3D (unequal subset sizes) and 2D (equal sizes)
    rng = np.random.default_rng(11)
    for nd, K in [(3, 5), (3, 7), (2, 9)]:
        pix = orc.subsets(nd, K)
        disagree = 0
        for _ in range(300):
            m = (rng.random(K ** nd) > rng.uniform(0.02, 0.5)).astype(np.uint8)
            want, fr = _fraction_rule(pix, m)
            assert orc.choose_subset(pix, m) == want
            disagree += int(np.argmax([int(m[p].sum()) for p in pix])) != want
        if nd == 3:
            assert disagree > 0   # the count rule would have failed here


def test_query_uses_the_subset_choice(orc):
    # The index query picks its subset by the same rule (query_point returns
    # the subset the query searched).
    rng = np.random.default_rng(5)
    vol = rng.random((12, 13, 11, 1)).astype(np.float32)
    mask = np.ones((12, 13, 11), np.uint8)
    mask[5:8, 5:8, 4:7] = 0
    ix = orc.Index(vol, mask, 5, 4, 2, key_bits=8)
    ms = [_mask_3d_k5(lambda i, j, k: i == 0), _mask_3d_k5(lambda i, j, k: j == 2 and k == 2)]
    ms += [(rng.random(125) > 0.3).astype(np.uint8) for _ in range(20)]
    m = np.stack(ms)
    t = rng.random((m.shape[0], 125, 1)).astype(np.float32)
    sub, _ = ix.query_point(t, m)
    _, _, _, _, sub2 = ix.query(vol, t, m)
    want = [_fraction_rule(ix.pix, mm)[0] for mm in m]
    assert sub[0] == 21 and sub[1] == 1
    assert list(sub) == want and list(sub2) == want


# Windows written out by hand from the reading of Section II.C's search: p is
# the first position whose key is >= the query key, lo = p - floor(W/2)
# clamped to [0, max(n - W, 0)], the window is [lo, min(lo + W, n)).
_KEYS1 = [3, 5, 5, 5, 9, 12, 12, 20, 31, 40]          # n = 10, one word


@pytest.mark.parametrize("q,W,p,lo", [
    (1, 4, 0, 0),      # below the first key: p = 0, window at the start
    (3, 4, 0, 0),      # equal to the first key
    (50, 4, 10, 6),    # above the last key: p = n, window at the end
    (40, 4, 9, 6),     # equal to the last key: lo = 7 clamped to n - W = 6
    (5, 4, 1, 0),      # a run of duplicates 5, 5, 5: p is its first position
    (5, 2, 1, 0),      # p - 1 = 0
    (6, 2, 4, 3),      # between the run and 9: p = 4
    (10, 4, 5, 3),     # mid-array between 9 and 12
    (12, 4, 5, 3),     # first of the run 12, 12
    (13, 4, 7, 5),     # after the run: p = 7 (key 20)
    (20, 5, 7, 5),     # odd W: floor(5/2) = 2
    (9, 1, 4, 4),      # W = 1: the lower-bound position itself
    (31, 3, 8, 7),     # odd W near the end: lo = 7 = n - W
    (9, 10, 4, 0),     # W = n: the whole array
    (9, 16, 4, 0),     # W > n: lo = 0, window [0, n)
])
def test_window_placement_hand_cases(orc, q, W, p, lo):
    keys = np.array(_KEYS1, np.uint64)
    assert orc.window(keys, q, W) == (p, lo)


def test_window_placement_two_word_keys(orc):
    # word 0 most significant: (1, 7) < (2, 0) < (2, 0) < (2, 5) < (3, 1)
    keys = np.array([[1, 7], [2, 0], [2, 0], [2, 5], [3, 1]], np.uint64)
    assert orc.window(keys, [2, 0], 2) == (1, 0)
    assert orc.window(keys, [2, 1], 2) == (3, 2)
    assert orc.window(keys, [1, 8], 2) == (1, 0)     # the low word decides within (1, .)
    assert orc.window(keys, [3, 2], 2) == (5, 3)
    assert orc.window(keys, [0, 2**64 - 1], 3) == (0, 0)
    # a high word of 2^63 and above compares unsigned
    keys = np.array([[5, 0], [2**63, 0], [2**64 - 1, 3]], np.uint64)
    assert orc.window(keys, [2**63 + 1, 0], 1) == (2, 2)


def test_index_query_windows_are_the_hand_rule(orc):
    # The index query's candidates are the union of the windows on its
    # curves: with L = 1 and W = 8 on a small index, every query's candidate
    # set is exactly 8 consecutive entries of the curve (or n of them), and
    # the query's own key, re-derived from query_point through key_of, has
    # its lower-bound position inside the window at offset floor(W/2) unless
    # the window was clamped at an end.
    vol, mask = _img(h=40, w=42, c=1, seed=9)
    K, W = 5, 8
    ix = orc.Index(vol, mask, K, 3, 1, key_bits=8, window=W)
    f = orc.front(mask)[::7]
    t, m = orc.extract(vol, mask, K, f)
    _, _, cand, nc, sub = ix.query(vol, t, m)
    _, ys = ix.query_point(t, m)
    R = 1 << ix.b
    for q in range(len(f)):
        s = sub[q]
        ids = ix.ids[s, 0]
        u = np.floor((ys[q] - ix.lo[s]) * (R - 1) / ix.span[s])
        v = np.clip(u, 0, R - 1).astype(np.uint32)
        qk = orc.key_of(v, ix.b, ix.curve)
        keys = ix.keys[s, 0]
        kint = [int(k[0]) for k in keys]
        p = int(np.searchsorted(np.array(kint, dtype=np.uint64), np.uint64(qk[0]), side="left"))
        lo = min(max(p - W // 2, 0), max(ix.n - W, 0))
        assert nc[q] == min(W, ix.n)
        assert np.array_equal(np.sort(cand[q, :nc[q]]), np.sort(ids[lo:lo + W]))


def test_more_curves_lower_acceleration_error(orc):
    """Table 3 trend: a larger candidate set lowers the acceleration error."""
    c1 = synth.config1()
    vol, mask = c1["volume"], c1["mask"]
    f = orc.front(mask)[::2]
    t, m = orc.extract(vol, mask, 9, f)
    d = orc.dictionary(mask, 9)
    b2, c2 = orc.brute(vol, mask.shape, 9, d, t, m)
    aes = []
    for L in (1, 4, 8):
        ix = orc.Index(vol, mask, 9, D=8, L=L, key_bits=12, window=32)
        bi, bc, *_ = ix.query(vol, t, m)
        assert np.all(bc >= c2)
        ok = c2 > 0
        aes.append(float(np.mean(np.sqrt(bc[ok]) / np.sqrt(c2[ok]) - 1)))
    assert aes[0] > aes[1] > aes[2]


# ------------------------------------------------------------------ inpainting loop
@pytest.mark.parametrize("order,mode", [("criminisi", "brute"), ("raster", "brute"),
                                        ("criminisi", "index")])
def test_inpaint_invariants(orc, order, mode):
    vol, mask = _img(h=30, w=32, c=2, seed=15, frac=0.06, holes=2)
    K = 5
    ix = orc.Index(vol, mask, K, D=6, L=3, key_bits=12, window=16) if mode == "index" else None
    out, mout, log = orc.inpaint(vol, mask, K, order=order, mode=mode, index=ix)
    assert np.all(mout == 1)
    assert log["iters"] == len(log["centre"]) > 0
    # replaying the logged copies on the input reproduces the output
    rv, rm = vol.copy(), mask.copy()
    H, W = mask.shape
    d = set(orc.dictionary(mask, K).tolist())
    for c, s in zip(log["centre"], log["source"]):
        assert int(s) in d
        cy, cx = divmod(int(c), W)
        sy, sx = divmod(int(s), W)
        for dy in range(-2, 3):
            for dx in range(-2, 3):
                y, x = cy + dy, cx + dx
                if 0 <= y < H and 0 <= x < W and not rm[y, x]:
                    rv[y, x] = rv[sy + dy, sx + dx]
                    rm[y, x] = 1
    assert np.array_equal(rv, out) and np.all(rm == 1)
    assert np.array_equal(out[mask == 1], vol[mask == 1])


def test_inpaint_constant_image_stays_constant(orc):
    vol = np.full((24, 24, 1), 0.75, np.float32)
    mask = np.ones((24, 24), np.uint8)
    mask[10:14, 9:15] = 0
    vol[mask == 0] = 0
    out, mout, log = orc.inpaint(vol, mask, 5)
    assert np.all(out == 0.75) and np.all(log["cost"] == 0.0)


def test_inpaint_single_pixel_hole_is_one_query(orc):
    vol, _ = _img(h=20, w=20, seed=16, frac=0.01, holes=1)
    mask = np.ones((20, 20), np.uint8)
    mask[9, 11] = 0
    vol[9, 11] = 0
    out, _, log = orc.inpaint(vol, mask, 5, order="raster")
    assert log["iters"] == 1
    c = orc.front(mask)[0]
    t, m = orc.extract(vol, mask, 5, [c])
    bi, bc = orc.brute(vol, mask.shape, 5, orc.dictionary(mask, 5), t, m)
    assert log["centre"][0] == c and log["source"][0] == bi[0] and log["cost"][0] == bc[0]


# ------------------------------------------------------------------ fill-order priority
# Closed forms on linear ramps, where the gradient by differences is exact:
# with the hole a half-plane, a front voxel's data term is the isophote's
# component along the boundary normal, and its confidence (first step) is the
# known fraction of its box.
def _ramp(shape, slopes, C=1, ch_scale=(1.0,)):
    grids = np.meshgrid(*[np.arange(s, dtype=np.float64) for s in shape], indexing="ij")
    base = sum(sl * g for sl, g in zip(slopes, grids))
    vol = np.stack([base * ch_scale[c % len(ch_scale)] for c in range(C)], -1)
    return vol.astype(np.float32)


@pytest.mark.parametrize("K", [5, 7, 9])
def test_priority_vertical_boundary(orc, K):
    # I = a x + b y, hole = columns right of x0: D = |b| (isophote (-b, a)
    # against the normal (0, -1)), C_p = (h + 1) / K away from the borders
    a, b = 0.25, -0.375
    h = K // 2
    H, W, x0 = 31, 29, 14
    vol = _ramp((H, W), (b, a))
    mask = np.ones((H, W), np.uint8)
    mask[:, x0 + 1:] = 0
    y = 15
    P, Cp = orc.priority(vol, mask, K, y * W + x0)
    assert Cp == (h + 1) / K
    assert P == ((h + 1) / K) * abs(b)
    # on the top row the box loses h rows; the normal ignores the border
    # (out of bounds counts as known) and the y-difference becomes one-sided
    P0, C0 = orc.priority(vol, mask, K, 0 * W + x0)
    assert C0 == (h + 1) ** 2 / K ** 2
    assert P0 == ((h + 1) ** 2 / K ** 2) * abs(b)


def test_priority_horizontal_boundary_multichannel(orc):
    # hole = rows below y0: D = |a| with a the x-slope of the channel mean
    K, h = 7, 3
    H, W, y0 = 25, 27, 11
    vol = _ramp((H, W), (0.5, 1.0), C=3, ch_scale=(0.25, 0.5, 0.75))   # mean scale 0.5
    mask = np.ones((H, W), np.uint8)
    mask[y0 + 1:, :] = 0
    P, Cp = orc.priority(vol, mask, K, y0 * W + 13)
    assert Cp == (h + 1) / K
    assert P == ((h + 1) / K) * 0.5


def test_priority_3d_half_space(orc):
    # I = c z + b y + a x, hole = x > x0: |grad I x n| with n = (0, 0, -1)
    # is sqrt(b^2 + c^2) = 5/8 for b = 3/8, c = 1/2
    K, h = 5, 2
    shape, x0 = (13, 12, 14), 6
    vol = _ramp(shape, (0.5, 0.375, 0.125))
    mask = np.ones(shape, np.uint8)
    mask[:, :, x0 + 1:] = 0
    p = (6 * shape[1] + 5) * shape[2] + x0
    P, Cp = orc.priority(vol, mask, K, p)
    assert Cp == (h + 1) / K
    assert P == ((h + 1) / K) * 0.625


def test_priority_confidence_is_box_sum_over_k_to_the_d(orc):
    # a later step: confidence values below 1 on some known voxels; C_p sums
    # the known in-bounds ones of the box and divides by K^d (not by the
    # known count), and unknown voxels contribute nothing
    K = 5
    H, W, x0 = 20, 20, 9
    vol = _ramp((H, W), (0.0, 1.0))
    mask = np.ones((H, W), np.uint8)
    mask[:, x0 + 1:] = 0
    conf = np.where(mask == 1, 1.0, 0.0)
    conf[8:13, x0 - 2:x0 + 1] = 0.5       # the known part of the box of (10, x0)
    conf[8:13, x0 + 1:x0 + 3] = 7.0       # unknown: must not count
    _, Cp = orc.priority(vol, mask, K, 10 * W + x0, conf=conf)
    assert Cp == (15 * 0.5) / 25
    # the data term does not see the confidence: the ramp's y-slope is 0
    P, _ = orc.priority(vol, mask, K, 10 * W + x0, conf=conf)
    assert P == 0.0


def test_priority_corner_uses_known_neighbours_only(orc):
    # known region = the quadrant y <= y0, x <= x0; the hole holds values far
    # off the ramp, so a difference that used an unknown neighbour would show.
    # At (y0, x0) both differences are one-sided (b and a) and the normal is
    # (-1, -1)/sqrt(2): D = |a - b| / sqrt(2); the box holds (h+1)^2 known
    K, h = 5, 2
    H, W, y0, x0 = 21, 23, 10, 12
    a, b = 0.75, -0.25
    vol = _ramp((H, W), (b, a))
    mask = np.zeros((H, W), np.uint8)
    mask[:y0 + 1, :x0 + 1] = 1
    vol[mask == 0] = 100.0
    P, Cp = orc.priority(vol, mask, K, y0 * W + x0)
    assert Cp == (h + 1) ** 2 / K ** 2
    assert P == pytest.approx(Cp * abs(a - b) / np.sqrt(2.0), rel=1e-15)


def test_query_imputation_is_the_ridge_least_squares_fit(orc):
    # the imputation solves (W_k^T W_k + I) a = W_k^T (x_k - mu_k); the same
    # fit is the plain least-squares solution of the stacked system
    # [W_k; I] a = [x_k - mu_k; 0], which numpy solves independently (SVD)
    import ctypes
    vol, mask = _img(h=44, w=42, c=3, seed=21)
    K = 5
    ix = orc.Index(vol, mask, K, D=6, L=2, key_bits=12, window=16)
    L = orc.lib()
    L.orc_query_point.restype = ctypes.c_int
    L.orc_query_point.argtypes = [ctypes.POINTER(orc.OrcIndex), ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p]
    rng = np.random.default_rng(4)
    cen = ix.dict[rng.choice(ix.n, 6, replace=False)]
    t, m = orc.extract(vol, mask, K, cen)
    C = vol.shape[-1]
    for q in range(len(cen)):
        mh = m[q].copy()
        mh[rng.random(mh.size) < 0.35] = 0
        yq = np.zeros(64)
        s = L.orc_query_point(ctypes.byref(ix.struct()), t[q].ctypes.data, mh.ctypes.data,
                              yq.ctypes.data)
        els = np.array([p * C + c for p in ix.pix[s] for c in range(C)])
        W = ix.bases[s].astype(np.float64)
        kn = np.repeat(mh[ix.pix[s]].astype(bool), C)
        x = np.clip(np.rint((t[q].reshape(-1)[els] - ix.vmin) * ix.qscale), 0, 255)
        mu = ix.sum[els] / ix.nsub
        D = W.shape[1]
        A = np.vstack([W[kn], np.eye(D)])
        rhs = np.concatenate([x[kn] - mu[kn], np.zeros(D)])
        a = np.linalg.lstsq(A, rhs, rcond=None)[0]
        ref = W[kn].T @ x[kn] + W[~kn].T @ (mu[~kn] + W[~kn] @ a)
        assert np.allclose(yq[:D], ref, rtol=1e-9, atol=1e-7), (q, yq[:D], ref)
