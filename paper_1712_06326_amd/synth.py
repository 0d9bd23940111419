"""Seeded synthetic workloads for the masked-L2 patch search.

This module only draws inputs: volumes, known-masks and image batches. It holds
none of the search method's arithmetic (no fill front, no cost, no keys) and
imports nothing from the rest of the package, so the CPU oracle's tests and the
GPU path can both consume exactly the same arrays.

Every generator takes an integer seed and uses numpy's PCG64 generator. Volumes
are float32 laid out [spatial..., C] with the channel innermost; masks are uint8
[spatial...] with 1 = known, 0 = missing. Missing voxels are set to 0.0 so that
no stale value can leak into a computation that is supposed to ignore them.

The stand-ins follow the paper's evaluation setting (natural colour images with
a missing region, Section II.I) and its motivating volume case (dictionaries of
more than 1e8 patches in 3D, Section I), without its image database.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng_for", "gradient_noise", "texture", "texture_rgb", "square_hole",
    "ellipse_mask", "config1", "config2", "config3", "config4", "config5",
    "small_image", "small_volume", "CONFIG_SEEDS",
]

CONFIG_SEEDS = {1: 1001, 2: 1002, 3: 1003, 4: 1004, 5: 1005}


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _fade(t):
    # quintic smoothstep 6t^5 - 15t^4 + 10t^3
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def gradient_noise(h: int, w: int, period: int, rng: np.random.Generator) -> np.ndarray:
    """Lattice gradient noise on an (h, w) grid with lattice spacing `period`.

    Random unit gradients sit on the lattice; each pixel blends the four corner
    dot products with the quintic fade. Output is float64 roughly in [-1, 1].
    """
    gh, gw = h // period + 2, w // period + 2
    ang = rng.uniform(0.0, 2.0 * np.pi, size=(gh, gw))
    gy, gx = np.sin(ang), np.cos(ang)
    y = (np.arange(h) + 0.5) / period
    x = (np.arange(w) + 0.5) / period
    iy = np.floor(y).astype(np.int64)
    ix = np.floor(x).astype(np.int64)
    fy = (y - iy)[:, None]
    fx = (x - ix)[None, :]
    iy2, ix2 = iy[:, None], ix[None, :]

    def dot(oy, ox):
        return gy[iy2 + oy, ix2 + ox] * (fy - oy) + gx[iy2 + oy, ix2 + ox] * (fx - ox)

    uy, ux = _fade(fy), _fade(fx)
    top = dot(0, 0) * (1 - ux) + dot(0, 1) * ux
    bot = dot(1, 0) * (1 - ux) + dot(1, 1) * ux
    return top * (1 - uy) + bot * uy


def _edges(h: int, w: int, count: int, rng: np.random.Generator) -> np.ndarray:
    out = np.zeros((h, w))
    yy, xx = np.mgrid[0:h, 0:w]
    for _ in range(count):
        th = rng.uniform(0.0, np.pi)
        py, px = rng.uniform(0, h), rng.uniform(0, w)
        amp = rng.uniform(-0.3, 0.3)
        side = (np.cos(th) * (yy - py) + np.sin(th) * (xx - px)) > 0
        out += amp * side
    return out


def _normalise(a: np.ndarray) -> np.ndarray:
    lo, hi = float(a.min()), float(a.max())
    if hi <= lo:
        return np.zeros_like(a, dtype=np.float32)
    return ((a - lo) / (hi - lo)).astype(np.float32)


def texture(h: int, w: int, rng: np.random.Generator, n_edges: int = 12) -> np.ndarray:
    """Four octaves of gradient noise (periods 64/32/16/8, amplitude 0.5^k)
    plus `n_edges` random straight step edges, min-max normalised to [0, 1]."""
    acc = np.zeros((h, w))
    for k, p in enumerate((64, 32, 16, 8)):
        acc += (0.5 ** k) * gradient_noise(h, w, p, rng)
    acc += _edges(h, w, n_edges, rng)
    return _normalise(acc)


def texture_rgb(h: int, w: int, c: int, rng: np.random.Generator) -> np.ndarray:
    """C correlated channels: 0.6 * shared field + 0.4 * an independent one."""
    base = texture(h, w, rng).astype(np.float64)
    chans = [_normalise(0.6 * base + 0.4 * texture(h, w, rng)) for _ in range(c)]
    return np.stack(chans, axis=-1).astype(np.float32)


def square_hole(h: int, w: int, y0: int, y1: int, x0: int, x1: int) -> np.ndarray:
    m = np.ones((h, w), dtype=np.uint8)
    m[y0:y1, x0:x1] = 0
    return m


def _ellipse_union(h, w, centres, axes, angles, scale):
    miss = np.zeros((h, w), dtype=bool)
    for (cy, cx), (a, b), th in zip(centres, axes, angles):
        a, b = a * scale, b * scale
        r = int(np.ceil(max(a, b))) + 1
        y0, y1 = max(0, int(cy) - r), min(h, int(cy) + r + 1)
        x0, x1 = max(0, int(cx) - r), min(w, int(cx) + r + 1)
        if y0 >= y1 or x0 >= x1:
            continue
        yy, xx = np.mgrid[y0:y1, x0:x1]
        dy, dx = yy - cy, xx - cx
        u = np.cos(th) * dx + np.sin(th) * dy
        v = -np.sin(th) * dx + np.cos(th) * dy
        miss[y0:y1, x0:x1] |= (u / a) ** 2 + (v / b) ** 2 <= 1.0
    return miss


def ellipse_mask(h: int, w: int, count: int, target: float, tol: float,
                 rng: np.random.Generator, axis_range=(10.0, 45.0)) -> np.ndarray:
    """Known-mask with `count` random elliptical blobs missing; the semi-axes
    are rescaled by bisection until the missing fraction is target +- tol."""
    centres = np.stack([rng.uniform(0, h, count), rng.uniform(0, w, count)], axis=1)
    axes = rng.uniform(axis_range[0], axis_range[1], size=(count, 2))
    angles = rng.uniform(0.0, np.pi, count)
    lo, hi = 0.05, 8.0
    miss = _ellipse_union(h, w, centres, axes, angles, 1.0)
    for _ in range(60):
        frac = miss.mean()
        if abs(frac - target) <= tol:
            break
        mid = 0.5 * (lo + hi)
        miss = _ellipse_union(h, w, centres, axes, angles, mid)
        if miss.mean() > target:
            hi = mid
        else:
            lo = mid
    return (~miss).astype(np.uint8)


def _apply_mask(vol: np.ndarray, mask: np.ndarray) -> np.ndarray:
    vol = np.ascontiguousarray(vol, dtype=np.float32)
    if vol.ndim == mask.ndim:
        vol[mask == 0] = 0.0
    else:
        vol[mask == 0, :] = 0.0
    return vol


def _pack(vol, mask, name, **extra):
    vol = np.ascontiguousarray(vol, dtype=np.float32)
    if vol.ndim == mask.ndim:
        vol = vol[..., None]
    d = dict(name=name, volume=vol, mask=np.ascontiguousarray(mask, dtype=np.uint8),
             shape=tuple(mask.shape), channels=int(vol.shape[-1]))
    d.update(extra)
    return d


def config1(seed: int = CONFIG_SEEDS[1]) -> dict:
    """256^2 grey texture, one 32x32 hole at [112,144)^2, 9x9 patches."""
    rng = rng_for(seed)
    img = texture(256, 256, rng)
    mask = square_hole(256, 256, 112, 144, 112, 144)
    return _pack(_apply_mask(img, mask), mask, "config1_256sq_gray_hole32_K9", K=9)


def config2(seed: int = CONFIG_SEEDS[2], size: int = 1024) -> dict:
    """1024^2 RGB, correlated channels, ~10% missing as 40 elliptical blobs,
    9x9x3 patches; index with D=8, 21-bit coordinates, 4 Morton curves, W=32."""
    rng = rng_for(seed)
    img = texture_rgb(size, size, 3, rng)
    scale = size / 1024.0
    mask = ellipse_mask(size, size, 40, 0.10, 0.002, rng,
                        axis_range=(10.0 * scale, 45.0 * scale))
    return _pack(_apply_mask(img, mask), mask, f"config2_{size}sq_rgb_blobs10_K9", K=9,
                 D=8, key_bits=21, n_curves=4, window=32, curve="morton")


def _gauss_blur3(vol, sigma):
    from scipy.ndimage import gaussian_filter
    return gaussian_filter(vol, sigma=sigma, mode="nearest")


def _sphere_mask(shape, frac, r_range, rng, start=None):
    miss = np.zeros(shape, dtype=bool) if start is None else start.copy()
    total = float(np.prod(shape))
    count = int(miss.sum())
    zz = np.arange(shape[0])
    yy = np.arange(shape[1])
    xx = np.arange(shape[2])
    while count / total < frac:
        r = rng.uniform(*r_range)
        c = [rng.uniform(0, s) for s in shape]
        lo = [max(0, int(c[i] - r) - 1) for i in range(3)]
        hi = [min(shape[i], int(c[i] + r) + 2) for i in range(3)]
        dz = (zz[lo[0]:hi[0]] - c[0])[:, None, None]
        dy = (yy[lo[1]:hi[1]] - c[1])[None, :, None]
        dx = (xx[lo[2]:hi[2]] - c[2])[None, None, :]
        sub = miss[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
        ball = dz * dz + dy * dy + dx * dx <= r * r
        count += int(np.count_nonzero(ball & ~sub))
        sub |= ball
    return miss


def _random_rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    return q * np.sign(np.diag(r))


def config3(seed: int = CONFIG_SEEDS[3], size: int = 256) -> dict:
    """256^3 tomogram: 60 random ellipsoids, Gaussian-blurred boundaries
    (sigma 1.5), noise sigma 0.02; ~5% missing as spherical voids; 7^3 patches."""
    rng = rng_for(seed)
    s = size / 256.0
    vol = np.zeros((size,) * 3, dtype=np.float32)
    g = np.arange(size, dtype=np.float32)
    for _ in range(60):
        ax = rng.uniform(8 * s, 48 * s, 3)
        rot = _random_rotation(rng)
        c = rng.uniform(0, size, 3)
        val = rng.uniform(0.2, 1.0)
        r = int(np.ceil(ax.max())) + 1
        lo = [max(0, int(c[i]) - r) for i in range(3)]
        hi = [min(size, int(c[i]) + r + 1) for i in range(3)]
        if any(lo[i] >= hi[i] for i in range(3)):
            continue
        dz = g[lo[0]:hi[0]][:, None, None] - c[0]
        dy = g[lo[1]:hi[1]][None, :, None] - c[1]
        dx = g[lo[2]:hi[2]][None, None, :] - c[2]
        q = 0.0
        for k in range(3):
            comp = rot[0, k] * dz + rot[1, k] * dy + rot[2, k] * dx
            q = q + (comp / ax[k]) ** 2
        sub = vol[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
        sub[q <= 1.0] = val
    vol = _gauss_blur3(vol, 1.5)
    vol = vol + rng.normal(0.0, 0.02, size=vol.shape).astype(np.float32)
    miss = _sphere_mask(vol.shape, 0.05, (4 * s, 16 * s), rng)
    mask = (~miss).astype(np.uint8)
    return _pack(_apply_mask(vol, mask), mask, f"config3_{size}cube_tomo_voids5_K7", K=7,
                 D=10, key_bits=8, n_curves=6, window=32, curve="hilbert")


def config4(seed: int = CONFIG_SEEDS[4], size: int = 512) -> dict:
    """512^3 layered-material phantom (uint16 phases converted to float32) with
    pores; ~2% missing as slabs plus spheres; 5^3 patches; 8-bit keys, 4 curves."""
    rng = rng_for(seed)
    s = size / 512.0
    phases = rng.integers(0, 65536, size=7).astype(np.float32)
    tilt = rng.uniform(0.0, 0.35)
    az = rng.uniform(0.0, 2 * np.pi)
    nrm = np.array([np.cos(tilt), np.sin(tilt) * np.sin(az), np.sin(tilt) * np.cos(az)])
    cuts = np.sort(rng.uniform(0.1, 0.9, 5)) * size
    vol = np.empty((size,) * 3, dtype=np.float32)
    g = np.arange(size, dtype=np.float64)
    proj_yx = nrm[1] * g[:, None] + nrm[2] * g[None, :]
    for z in range(size):
        p = nrm[0] * z + proj_yx
        vol[z] = phases[np.searchsorted(cuts, p)]
    pores = _sphere_mask(vol.shape, 0.01, (2 * s, 12 * s), rng)
    vol[pores] = phases[6]
    miss = np.zeros(vol.shape, dtype=bool)
    for _ in range(2):
        axis = int(rng.integers(0, 3))
        th = int(rng.integers(2, 7))
        pos = int(rng.integers(0, size - th))
        sl = [slice(None)] * 3
        sl[axis] = slice(pos, pos + th)
        ext = [slice(int(rng.integers(0, size // 2)), None) for _ in range(3)]
        ext[axis] = sl[axis]
        miss[tuple(ext)] = True
    miss = _sphere_mask(vol.shape, 0.02, (3 * s, 12 * s), rng, start=miss)
    mask = (~miss).astype(np.uint8)
    return _pack(_apply_mask(vol, mask), mask, f"config4_{size}cube_phantom_u16_K5", K=5,
                 D=8, key_bits=8, n_curves=4, window=32, curve="morton")


def config5(seed: int = CONFIG_SEEDS[5], n_images: int = 64, side_range=(256, 2048)) -> list:
    """Batch of images with sides U{256..2048}, 1-3 channels, 5-15% missing."""
    rng = rng_for(seed)
    out = []
    for i in range(n_images):
        h = int(rng.integers(side_range[0], side_range[1] + 1))
        w = int(rng.integers(side_range[0], side_range[1] + 1))
        c = int(rng.integers(1, 4))
        frac = float(rng.uniform(0.05, 0.15))
        sub = rng_for(int(rng.integers(0, 2**31)))
        img = texture_rgb(h, w, c, sub)
        sc = min(h, w) / 1024.0
        mask = ellipse_mask(h, w, 40, frac, 0.004, sub,
                            axis_range=(max(3.0, 10.0 * sc), max(6.0, 45.0 * sc)))
        out.append(_pack(_apply_mask(img, mask), mask, f"img{i}_{h}x{w}x{c}", K=9))
    return out


def small_image(h: int, w: int, c: int, seed: int, holes: int = 3, frac: float = 0.1) -> dict:
    """Small textured image with a few elliptical holes (test inputs)."""
    rng = rng_for(seed)
    img = texture_rgb(h, w, c, rng) if c > 1 else texture(h, w, rng)
    sc = min(h, w) / 64.0
    mask = ellipse_mask(h, w, holes, frac, 0.01, rng, axis_range=(2.0 * sc, 6.0 * sc))
    return _pack(_apply_mask(img, mask), mask, f"small_{h}x{w}x{c}_s{seed}")


def small_volume(n: int, seed: int, frac: float = 0.05, c: int = 1) -> dict:
    """Small blurred-blob volume with spherical voids (test inputs)."""
    rng = rng_for(seed)
    vol = rng.uniform(0, 1, size=(n, n, n, c)).astype(np.float32)
    from scipy.ndimage import gaussian_filter
    vol = gaussian_filter(vol, sigma=(1.2, 1.2, 1.2, 0)).astype(np.float32)
    miss = _sphere_mask((n, n, n), frac, (1.5, 3.0), rng)
    mask = (~miss).astype(np.uint8)
    vol[mask == 0, :] = 0.0
    return _pack(vol, mask, f"smallvol_{n}cube_c{c}_s{seed}")
