"""Seeded synthetic inputs shaped like the workloads the GGDT path is measured on.

This module holds no distance-transform arithmetic: it only draws images, soft
masks, spacings and loss weights.  Both the HIP path and the CPU oracle consume
what it returns, byte for byte.

Recipes (the paper names no dataset; these stand in for its "3D volume data"):
  * blurred noise: uniform[0,1) noise, separable Gaussian blur (truncated at
    4 sigma, reflect boundary);
  * 2D ellipses: centre uniform in the image, semi-axes U[W/32, W/6], rotation
    U[0, pi), an additive constant U[jump range] per channel inside;
  * 3D ellipsoids: centre uniform, semi-axes U[8, 64] voxels times a size scale
    (min(shape) / 256), random rotation, additive constant U[0.2, 1.0] inside;
  * hard-seed masks: 1 everywhere, 0 on a seeded square/cube or on seeded points;
  * soft masks: sigmoid(3 z), z = blurred noise standardised to mean 0, std 1.
Every configuration uses its own seed, 220800000 + config number, and named
sub-streams so that changing one draw never shifts another.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

SEED_BASE = 220800000


def rng_for(seed: int, stream: str) -> np.random.Generator:
    """Independent generator for a named sub-stream of a seed."""
    key = [seed] + [ord(ch) for ch in stream]
    return np.random.default_rng(key)


def blurred_noise(shape, sigma, rng) -> np.ndarray:
    x = rng.random(shape, dtype=np.float64)
    x = ndimage.gaussian_filter(x, sigma=sigma, mode="reflect", truncate=4.0)
    return x


def _rotation_3d(rng) -> np.ndarray:
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def add_ellipses_2d(img: np.ndarray, n: int, jump, rng) -> None:
    """img: (C, H, W), modified in place."""
    C, H, W = img.shape
    yy, xx = np.mgrid[0:H, 0:W]
    for _ in range(n):
        cy, cx = rng.uniform(0, H), rng.uniform(0, W)
        ay, ax = rng.uniform(W / 32, W / 6), rng.uniform(W / 32, W / 6)
        th = rng.uniform(0, np.pi)
        amp = rng.uniform(jump[0], jump[1], size=C)
        r = int(np.ceil(max(ay, ax))) + 1
        y0, y1 = max(0, int(cy) - r), min(H, int(cy) + r + 1)
        x0, x1 = max(0, int(cx) - r), min(W, int(cx) + r + 1)
        if y0 >= y1 or x0 >= x1:
            continue
        dy = yy[y0:y1, x0:x1] - cy
        dx = xx[y0:y1, x0:x1] - cx
        u = np.cos(th) * dy + np.sin(th) * dx
        w = -np.sin(th) * dy + np.cos(th) * dx
        inside = (u / ay) ** 2 + (w / ax) ** 2 <= 1.0
        for c in range(C):
            img[c, y0:y1, x0:x1][inside] += amp[c]


def add_ellipsoids_3d(img: np.ndarray, n: int, jump, axes, rng) -> None:
    """img: (C, D, H, W), modified in place."""
    C = img.shape[0]
    shape = img.shape[1:]
    for _ in range(n):
        c0 = np.array([rng.uniform(0, s) for s in shape])
        semi = rng.uniform(axes[0], axes[1], size=3)
        R = _rotation_3d(rng)
        amp = rng.uniform(jump[0], jump[1], size=C)
        r = int(np.ceil(semi.max())) + 1
        lo = [max(0, int(c0[i]) - r) for i in range(3)]
        hi = [min(shape[i], int(c0[i]) + r + 1) for i in range(3)]
        if any(lo[i] >= hi[i] for i in range(3)):
            continue
        grid = np.stack(np.meshgrid(*[np.arange(lo[i], hi[i]) - c0[i] for i in range(3)], indexing="ij"), -1)
        local = grid @ R
        inside = ((local / semi) ** 2).sum(-1) <= 1.0
        for c in range(C):
            img[c, lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]][inside] += amp[c]


def box_seed_mask(shape, size, rng) -> np.ndarray:
    """1 everywhere, 0 inside one axis-aligned box of side `size` at a seeded place."""
    m = np.ones(shape, dtype=np.float32)
    sl = []
    for s in shape:
        side = min(size, s)
        o = int(rng.integers(0, s - side + 1))
        sl.append(slice(o, o + side))
    m[tuple(sl)] = 0.0
    return m


def point_seed_mask(shape, count, rng) -> np.ndarray:
    m = np.ones(shape, dtype=np.float32)
    flat = rng.choice(int(np.prod(shape)), size=min(count, int(np.prod(shape))), replace=False)
    m.reshape(-1)[flat] = 0.0
    return m


def soft_mask(shape, sigma, rng) -> np.ndarray:
    z = blurred_noise(shape, sigma, rng)
    z = (z - z.mean()) / max(z.std(), 1e-12)
    return (1.0 / (1.0 + np.exp(-3.0 * z))).astype(np.float32)


def image_2d(shape_hw, C, sigma, n_ellipses, seed, jump=(0.3, 0.8)) -> np.ndarray:
    rng = rng_for(seed, "image")
    img = np.stack([blurred_noise(shape_hw, sigma, rng) for _ in range(C)])
    if n_ellipses:
        add_ellipses_2d(img, n_ellipses, jump, rng_for(seed, "ellipses"))
    return img.astype(np.float32)


def volume_3d(shape_dhw, C, sigma, n_ellipsoids, seed, jump=(0.2, 1.0)) -> np.ndarray:
    rng = rng_for(seed, "image")
    img = np.stack([blurred_noise(shape_dhw, sigma, rng) for _ in range(C)])
    scale = min(shape_dhw) / 256.0
    if n_ellipsoids:
        add_ellipsoids_3d(img, n_ellipsoids, jump, (8 * scale, 64 * scale), rng_for(seed, "ellipsoids"))
    return img.astype(np.float32)


# ---------------------------------------------------------------- workloads

def config1(lam: float, seed: int = SEED_BASE + 1) -> dict:
    """2D 128x128, C=1, blurred noise sigma 2, 8x8 hard seed square, 2 iterations."""
    img = image_2d((128, 128), 1, 2.0, 0, seed)
    mask = box_seed_mask((128, 128), 8, rng_for(seed, "mask"))
    return dict(image=img, mask=mask, spacing=(1.0, 1.0), v=1e10, lam=float(lam), iterations=2, seed=seed,
                name=f"2d-128x128-c1-lam{lam:g}")


def config2(lam: float, seed: int = SEED_BASE + 2, size: int = 2048) -> dict:
    """2D 2048x2048, C=3, noise sigma 4 plus 6 ellipses, 16 seed pixels, 2 iterations."""
    img = image_2d((size, size), 3, 4.0, 6, seed)
    mask = point_seed_mask((size, size), 16, rng_for(seed, "mask"))
    return dict(image=img, mask=mask, spacing=(1.0, 1.0), v=1e10, lam=float(lam), iterations=2, seed=seed,
                name=f"2d-{size}x{size}-c3-lam{lam:g}")


def config3(seed: int = SEED_BASE + 3, size: int = 256) -> dict:
    """3D 256^3, C=1, noise sigma 3 plus 10 ellipsoids, spacing (1, 1, 2.5), 12^3 seed cube,
    lambda 1, 4 iterations."""
    img = volume_3d((size, size, size), 1, 3.0, 10, seed)
    mask = box_seed_mask((size, size, size), 12, rng_for(seed, "mask"))
    return dict(image=img, mask=mask, spacing=(1.0, 1.0, 2.5), v=1e10, lam=1.0, iterations=4, seed=seed,
                name=f"3d-{size}^3-c1-lam1")


def config4(seed: int = SEED_BASE + 4, n3d: int = 48, n2d: int = 16) -> list:
    """Ragged batch: 3D volumes U[64,192] x U[64,192] x U[64,96], 2D images U[256,1024]^2,
    per-instance lambda U[0,1], spacing U[0.5,3] per axis, 1-32 point seeds, 2-4 iterations."""
    rng = rng_for(seed, "batch")
    out = []
    for i in range(n3d + n2d):
        sub = seed * 1000 + i
        lam = float(np.float32(rng.uniform(0.0, 1.0)))
        iters = int(rng.integers(2, 5))
        nseed = int(rng.integers(1, 33))
        if i < n3d:
            shape = (int(rng.integers(64, 193)), int(rng.integers(64, 193)), int(rng.integers(64, 97)))
            sp = tuple(float(np.float32(s)) for s in rng.uniform(0.5, 3.0, size=3))
            img = volume_3d(shape, 1, 3.0, 10, sub)
        else:
            shape = (int(rng.integers(256, 1025)), int(rng.integers(256, 1025)))
            sp = tuple(float(np.float32(s)) for s in rng.uniform(0.5, 3.0, size=2))
            img = image_2d(shape, 1, 2.0, 0, sub)
        mask = point_seed_mask(shape, nseed, rng_for(sub, "mask"))
        out.append(dict(image=img, mask=mask, spacing=sp, v=1e10, lam=lam, iterations=iters, seed=sub,
                        name=f"inst{i}-{'x'.join(map(str, shape))}"))
    return out


def config5(seed: int = SEED_BASE + 5, size: int = 128, batch: int = 4) -> list:
    """Batch of 3D 128^3 volumes (config-3 recipe scaled), lambda 0.7, 3 iterations, soft mask
    sigmoid(3 z), v = 10, loss weights W ~ N(0, 1)."""
    out = []
    for b in range(batch):
        sub = seed * 1000 + b
        img = volume_3d((size, size, size), 1, 3.0, 10, sub)
        mask = soft_mask((size, size, size), 3.0, rng_for(sub, "softmask"))
        weight = rng_for(sub, "weight").standard_normal((size, size, size)).astype(np.float32)
        out.append(dict(image=img, mask=mask, spacing=(1.0, 1.0, 2.5), v=10.0, lam=0.7, iterations=3,
                        weight=weight, seed=sub, name=f"vol{b}-{size}^3"))
    return out


def small_case(shape, C=1, seed=0, lam=0.5, iterations=2, spacing=None, soft=False, v=1e10) -> dict:
    """Small random instance for parity tests: blurred noise (+ blobs), seeds or soft mask."""
    nd = len(shape)
    rng = rng_for(seed, "small")
    if nd == 2:
        img = image_2d(shape, C, 1.5, 2, seed)
    else:
        img = volume_3d(shape, C, 1.5, 3, seed)
    if soft:
        mask = soft_mask(shape, 1.5, rng_for(seed, "softmask"))
    else:
        mask = point_seed_mask(shape, int(rng.integers(1, 5)), rng_for(seed, "mask"))
    if spacing is None:
        spacing = tuple(float(np.float32(s)) for s in rng.uniform(0.5, 3.0, size=nd))
    return dict(image=img, mask=mask, spacing=tuple(spacing), v=float(v), lam=float(np.float32(lam)),
                iterations=int(iterations), seed=seed, name=f"small-{'x'.join(map(str, shape))}-c{C}")
