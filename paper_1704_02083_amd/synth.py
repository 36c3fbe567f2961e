"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no part of the segmentation method: it only draws images.
Both the GPU library's tests/benchmark and the CPU oracle consume its output.

Workloads (the paper's NLST whole-slide images and BSD500 photos are not
available; these stand in for them):
  * ``voronoi_blur``      256x256 mosaic of 24 random Voronoi regions with
                          uniform random colours, 3x3 box blur, N(0, 8^2) noise.
  * ``voronoi_gradient``  BSD500-shaped 481x321 / 321x481 mosaics of 30..120
                          regions with linear colour gradients, N(0, 6^2) noise.
  * ``he_tile``           H&E-like tissue: grey background on the 30 % (or
                          chosen) fraction of lowest Perlin mask, pink stroma,
                          purple elliptical nuclei at 1 per 400 px^2 of tissue.
"""
from __future__ import annotations

import numpy as np


def _voronoi_assign(W: int, H: int, sites: np.ndarray) -> np.ndarray:
    """Index of the nearest site (Euclidean) for every pixel."""
    from scipy.spatial import cKDTree
    ys, xs = np.mgrid[0:H, 0:W]
    _, idx = cKDTree(sites).query(np.stack([xs.ravel(), ys.ravel()], 1).astype(np.float64), workers=-1)
    return idx.reshape(H, W).astype(np.int32)


def _box3(img: np.ndarray) -> np.ndarray:
    """Integer 3x3 box filter with edge replication, rounded to nearest."""
    p = np.pad(img.astype(np.int32), ((1, 1), (1, 1), (0, 0)), mode="edge")
    H, W = img.shape[:2]
    s = np.zeros(img.shape, np.int32)
    for dy in range(3):
        for dx in range(3):
            s += p[dy:dy + H, dx:dx + W]
    return (s + 4) // 9


def _noise(rng: np.random.Generator, img: np.ndarray, sigma: float) -> np.ndarray:
    n = np.rint(rng.normal(0.0, sigma, size=img.shape))
    return np.clip(img + n, 0, 255).astype(np.uint8)


def voronoi_blur(W: int = 256, H: int = 256, regions: int = 24, sigma: float = 8.0,
                 seed: int = 1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    sites = rng.uniform(0, [W, H], size=(regions, 2))
    cols = rng.integers(0, 256, size=(regions, 3))
    img = cols[_voronoi_assign(W, H, sites)]
    img = _box3(img)
    return _noise(rng, img, sigma)


def voronoi_gradient(W: int = 481, H: int = 321, seed: int = 1000, sigma: float = 6.0,
                     regions: tuple[int, int] = (30, 120)) -> np.ndarray:
    rng = np.random.default_rng(seed)
    nreg = int(rng.integers(regions[0], regions[1] + 1))
    sites = rng.uniform(0, [W, H], size=(nreg, 2))
    c0 = rng.uniform(0, 255, size=(nreg, 3))
    g = rng.uniform(-0.5, 0.5, size=(nreg, 3, 2))
    idx = _voronoi_assign(W, H, sites)
    ys, xs = np.mgrid[0:H, 0:W]
    dx = xs - sites[idx, 0]
    dy = ys - sites[idx, 1]
    img = c0[idx] + g[idx, :, 0] * dx[..., None] + g[idx, :, 1] * dy[..., None]
    img = np.clip(np.rint(img), 0, 255)
    return _noise(rng, img, sigma)


def batch_images(n: int = 200, seed0: int = 1000) -> list[np.ndarray]:
    """The batched workload: half 481x321 (W x H), half 321x481."""
    out = []
    for i in range(n):
        if i < n // 2:
            out.append(voronoi_gradient(481, 321, seed=seed0 + i))
        else:
            out.append(voronoi_gradient(321, 481, seed=seed0 + i))
    return out


# ----------------------------------------------------------------- H&E tiles

def _perlin(W: int, H: int, cell: int, rng: np.random.Generator) -> np.ndarray:
    """Gradient ("improved") Perlin noise on a lattice of the given cell size,
    evaluated cell by cell with broadcasting."""
    gw, gh = -(-W // cell) + 1, -(-H // cell) + 1
    ang = rng.uniform(0, 2 * np.pi, size=(gh, gw))
    gxv, gyv = np.cos(ang), np.sin(ang)
    t = np.arange(cell, dtype=np.float64) / cell
    tx = t[None, None, None, :]
    ty = t[None, :, None, None]

    def corner(dy, dx):
        return (gxv[dy:dy + gh - 1, dx:dx + gw - 1][:, None, :, None],
                gyv[dy:dy + gh - 1, dx:dx + gw - 1][:, None, :, None])

    def fade(v):
        return v * v * v * (v * (v * 6 - 15) + 10)

    g00, g10, g01, g11 = corner(0, 0), corner(0, 1), corner(1, 0), corner(1, 1)
    n00 = g00[0] * tx + g00[1] * ty
    n10 = g10[0] * (tx - 1) + g10[1] * ty
    n01 = g01[0] * tx + g01[1] * (ty - 1)
    n11 = g11[0] * (tx - 1) + g11[1] * (ty - 1)
    u, v = fade(tx), fade(ty)
    out = (n00 * (1 - u) + n10 * u) * (1 - v) + (n01 * (1 - u) + n11 * u) * v
    return out.reshape((gh - 1) * cell, (gw - 1) * cell)[:H, :W]


def _fbm(W: int, H: int, cell: int, rng: np.random.Generator, octaves: int = 3) -> np.ndarray:
    out = np.zeros((H, W))
    amp = 1.0
    for o in range(octaves):
        c = max(cell >> o, 4)
        out += amp * _perlin(W, H, c, rng)
        amp *= 0.5
    return out


def he_tile(W: int = 4096, H: int = 4096, seed: int = 3, background: float = 0.30,
            nucleus_area: float = 400.0) -> np.ndarray:
    """H&E-like tile: grey background, pink stroma, purple nuclei."""
    rng = np.random.default_rng(seed)
    bg_mask = _fbm(W, H, 512, rng)
    thr = np.quantile(bg_mask, background)
    bg = bg_mask <= thr
    stroma_mask = _fbm(W, H, 128, rng)
    img = np.empty((H, W, 3), np.int32)
    # tissue base: pale pink/lilac, deeper pink where the stroma mask is high
    tissue_base = np.array([200, 160, 200])
    stroma = np.array([220, 150, 190])
    w = np.clip((stroma_mask + 0.2) * 2.5, 0, 1)[..., None]
    img[:] = np.rint(tissue_base * (1 - w) + stroma * w).astype(np.int32)
    img += rng.integers(-15, 16, size=(H, W, 3))
    grey = rng.integers(230, 246, size=(H, W))
    img[bg] = grey[bg][:, None]
    # nuclei: Poisson count over the tissue area, rejection of background centres
    tissue_px = int((~bg).sum())
    n_nuc = rng.poisson(tissue_px / nucleus_area)
    cx = rng.uniform(0, W, size=int(n_nuc * 1.0 / max(1e-9, 1 - background)) + 16)
    cy = rng.uniform(0, H, size=cx.shape[0])
    keep = ~bg[cy.astype(np.int64).clip(0, H - 1), cx.astype(np.int64).clip(0, W - 1)]
    cx, cy = cx[keep][:n_nuc], cy[keep][:n_nuc]
    n = cx.shape[0]
    ax = rng.uniform(3, 8, size=n)
    ay = rng.uniform(3, 8, size=n)
    th = rng.uniform(0, np.pi, size=n)
    base = np.array([90, 60, 140])[None, :] + rng.integers(-20, 21, size=(n, 3))
    for i in range(n):
        r = int(np.ceil(max(ax[i], ay[i])))
        x0, x1 = max(int(cx[i]) - r, 0), min(int(cx[i]) + r + 1, W)
        y0, y1 = max(int(cy[i]) - r, 0), min(int(cy[i]) + r + 1, H)
        if x0 >= x1 or y0 >= y1:
            continue
        yy, xx = np.mgrid[y0:y1, x0:x1]
        dx, dy = xx + 0.5 - cx[i], yy + 0.5 - cy[i]
        c, s = np.cos(th[i]), np.sin(th[i])
        u = (dx * c + dy * s) / ax[i]
        v = (-dx * s + dy * c) / ay[i]
        m = u * u + v * v <= 1.0
        patch = img[y0:y1, x0:x1]
        patch[m] = base[i] + rng.integers(-6, 7, size=(int(m.sum()), 3))
    return np.clip(img, 0, 255).astype(np.uint8)


def flat_mosaic(W: int, H: int, cell: int, seed: int = 0) -> np.ndarray:
    """Grid-aligned flat mosaic with distinct colours per cell (no noise)."""
    rng = np.random.default_rng(seed)
    gx, gy = -(-W // cell), -(-H // cell)
    cols = rng.permutation(256 ** 3 // 4099)[: gx * gy] * 4099
    rgb = np.stack([(cols >> 16) & 255, (cols >> 8) & 255, cols & 255], -1).astype(np.uint8)
    ys, xs = np.mgrid[0:H, 0:W]
    return rgb[(ys // cell) * gx + xs // cell]
