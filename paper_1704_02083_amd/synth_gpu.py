"""Whole-slide-scale synthetic H&E images generated with torch on the GPU.

Holds none of the segmentation method: it only draws images.  Every random
quantity is a counter-based hash (SplitMix64 finaliser) of (seed, stream,
coordinates), so any row band of the slide can be drawn independently and
the bands join seamlessly:

  * background: grey U{230..245} per pixel where a Perlin fBm mask (lattice
    512 px, 3 octaves) is below its `background` quantile;
  * tissue: a lilac base (200, 160, 200) blended towards pink stroma
    (220, 150, 190) by a second fBm mask (lattice 128 px), +-15 per channel;
  * nuclei: one per 20 x 20 px cell of tissue (1 per 400 px^2), an ellipse
    with semi-axes U[3, 8] px and random angle, centre uniform in the cell,
    colour (90, 60, 140) +- 20 per nucleus and +-6 per pixel.
The image stands in for the paper's NLST whole-slide images.
"""
from __future__ import annotations

import math

import torch

_M1 = 0xBF58476D1CE4E5B9 - (1 << 64)
_M2 = 0x94D049BB133111EB - (1 << 64)
_G = 0x9E3779B97F4A7C15 - (1 << 64)


def _mix(z: torch.Tensor) -> torch.Tensor:
    """SplitMix64 finaliser on int64 tensors (wrapping arithmetic)."""
    z = z + _G
    z = (z ^ ((z >> 30) & ((1 << 34) - 1))) * _M1
    z = (z ^ ((z >> 27) & ((1 << 37) - 1))) * _M2
    return z ^ ((z >> 31) & ((1 << 33) - 1))


def _hash(seed: int, stream: int, a: torch.Tensor, b: torch.Tensor, c: int = 0) -> torch.Tensor:
    z = _mix(torch.as_tensor(seed * 1000003 + stream, dtype=torch.int64, device=a.device) + a * 0x1F3D5B79)
    z = _mix(z + b * 0x2545F491 + c)
    return z


def _unit(h: torch.Tensor) -> torch.Tensor:
    """Uniform [0, 1) float32 from the top 24 bits of a hash."""
    return ((h >> 40) & 0xFFFFFF).to(torch.float32) / float(1 << 24)


def _perlin(xs: torch.Tensor, ys: torch.Tensor, cell: int, seed: int, stream: int) -> torch.Tensor:
    """Gradient noise at pixel columns xs (W,) and rows ys (H,) -> (H, W)."""
    fx = xs.to(torch.float32) / cell
    fy = ys.to(torch.float32) / cell
    ix, iy = torch.floor(fx).to(torch.int64), torch.floor(fy).to(torch.int64)
    tx, ty = (fx - ix)[None, :], (fy - iy)[:, None]

    def grad(dx, dy):
        ang = _unit(_hash(seed, stream, (ix + dx)[None, :], (iy + dy)[:, None])) * (2 * math.pi)
        return torch.cos(ang), torch.sin(ang)

    def fade(t):
        return t * t * t * (t * (t * 6 - 15) + 10)

    g00, g10, g01, g11 = grad(0, 0), grad(1, 0), grad(0, 1), grad(1, 1)
    n00 = g00[0] * tx + g00[1] * ty
    n10 = g10[0] * (tx - 1) + g10[1] * ty
    n01 = g01[0] * tx + g01[1] * (ty - 1)
    n11 = g11[0] * (tx - 1) + g11[1] * (ty - 1)
    u, v = fade(tx), fade(ty)
    return (n00 * (1 - u) + n10 * u) * (1 - v) + (n01 * (1 - u) + n11 * u) * v


def _fbm(xs, ys, cell, seed, stream, octaves=3):
    out = torch.zeros((ys.numel(), xs.numel()), dtype=torch.float32, device=xs.device)
    amp = 1.0
    for o in range(octaves):
        out += amp * _perlin(xs, ys, max(cell >> o, 4), seed, stream * 16 + o)
        amp *= 0.5
    return out


def background_threshold(W: int, H: int, seed: int, background: float, device) -> float:
    """The `background` quantile of the background mask, from a 1/16
    subsample of the slide."""
    xs = torch.arange(0, W, 16, device=device)
    ys = torch.arange(0, H, 16, device=device)
    m = _fbm(xs, ys, 512, seed, 1).ravel()
    if m.numel() > (1 << 24):
        m = m[:: (m.numel() >> 24) + 1]
    return float(torch.quantile(m, background).item())


def he_band(W: int, y0: int, y1: int, seed: int, thresh: float, device) -> torch.Tensor:
    """Rows [y0, y1) of the slide as (y1 - y0, W, 3) uint8."""
    xs = torch.arange(W, device=device)
    ys = torch.arange(y0, y1, device=device)
    bg = _fbm(xs, ys, 512, seed, 1) <= thresh
    w = torch.clamp((_fbm(xs, ys, 128, seed, 2) + 0.2) * 2.5, 0, 1)[..., None]
    base = torch.tensor([200.0, 160.0, 200.0], device=device)
    stroma = torch.tensor([220.0, 150.0, 190.0], device=device)
    img = torch.round(base * (1 - w) + stroma * w)
    X, Y = xs[None, :].expand(len(ys), W), ys[:, None].expand(len(ys), W)
    for ch in range(3):
        img[..., ch] += (_hash(seed, 3, X, Y, ch) % 31 - 15).to(torch.float32)
    # nuclei: one per 20 x 20 cell with its centre anywhere in the cell; the
    # parameters are drawn per cell, every pixel tests the nuclei of the 3 x 3
    # cells around its own (the first hit in a fixed order wins)
    c0y, c1y = y0 // 20 - 1, (y1 - 1) // 20 + 2
    ncw = (W - 1) // 20 + 3
    ccx = torch.arange(-1, ncw - 1, device=device)[None, :]
    ccy = torch.arange(c0y, c1y, device=device)[:, None]
    hc = [_hash(seed, 4, ccx, ccy, q) for q in range(6)]
    cax = 3 + 5 * _unit(hc[0])
    cay = 3 + 5 * _unit(hc[1])
    cth = math.pi * _unit(hc[2])
    cnx = ccx.to(torch.float32) * 20 + 20 * _unit(hc[3])
    cny = ccy.to(torch.float32) * 20 + 20 * _unit(hc[4])
    ctis = _fbm_points(cnx, cny, seed) > thresh
    ccol = torch.stack([90 + (hc[5] % 41 - 20), 60 + ((hc[5] >> 8) % 41 - 20),
                        140 + ((hc[5] >> 16) % 41 - 20)], -1).to(torch.float32)
    nuc = torch.zeros(X.shape, dtype=torch.bool, device=device)
    ncol = torch.zeros(X.shape + (3,), dtype=torch.float32, device=device)
    px, py = X.to(torch.float32) + 0.5, Y.to(torch.float32) + 0.5
    for oy in (-1, 0, 1):
        for ox in (-1, 0, 1):
            iy = Y // 20 + oy - c0y
            ix = X // 20 + ox + 1
            dx, dy = px - cnx[iy, ix], py - cny[iy, ix]
            c, s = torch.cos(cth[iy, ix]), torch.sin(cth[iy, ix])
            u = (dx * c + dy * s) / cax[iy, ix]
            v = (-dx * s + dy * c) / cay[iy, ix]
            hit = ((u * u + v * v) <= 1.0) & ctis[iy, ix] & ~nuc
            ncol = torch.where(hit[..., None], ccol[iy, ix], ncol)
            nuc |= hit
    nuc &= ~bg
    for ch in range(3):
        pn = (_hash(seed, 5, X, Y, ch) % 13 - 6).to(torch.float32)
        img[..., ch] = torch.where(nuc, ncol[..., ch] + pn, img[..., ch])
    grey = (230 + _hash(seed, 6, X, Y) % 16).to(torch.float32)
    img = torch.where(bg[..., None], grey[..., None], img)
    return torch.clamp(img, 0, 255).to(torch.uint8)


def _fbm_points(px: torch.Tensor, py: torch.Tensor, seed: int) -> torch.Tensor:
    """The background fBm at arbitrary points (same lattice as _fbm)."""
    out = torch.zeros_like(px)
    amp = 1.0
    for o in range(3):
        cell = max(512 >> o, 4)
        stream = 16 + o
        fx, fy = px / cell, py / cell
        ix, iy = torch.floor(fx).to(torch.int64), torch.floor(fy).to(torch.int64)
        tx, ty = fx - ix, fy - iy

        def grad(dx, dy):
            ang = _unit(_hash(seed, stream, ix + dx, iy + dy)) * (2 * math.pi)
            return torch.cos(ang), torch.sin(ang)

        def fade(t):
            return t * t * t * (t * (t * 6 - 15) + 10)

        g00, g10, g01, g11 = grad(0, 0), grad(1, 0), grad(0, 1), grad(1, 1)
        n00 = g00[0] * tx + g00[1] * ty
        n10 = g10[0] * (tx - 1) + g10[1] * ty
        n01 = g01[0] * tx + g01[1] * (ty - 1)
        n11 = g11[0] * (tx - 1) + g11[1] * (ty - 1)
        u, v = fade(tx), fade(ty)
        out += amp * ((n00 * (1 - u) + n10 * u) * (1 - v) + (n01 * (1 - u) + n11 * u) * v)
        amp *= 0.5
    return out


def he_slide(W: int, H: int, seed: int = 4, background: float = 0.4, device="cuda",
             band: int = 1024) -> torch.Tensor:
    """The whole slide as an (H, W, 3) uint8 tensor on `device`."""
    thresh = background_threshold(W, H, seed, background, device)
    out = torch.empty((H, W, 3), dtype=torch.uint8, device=device)
    for y0 in range(0, H, band):
        y1 = min(H, y0 + band)
        out[y0:y1] = he_band(W, y0, y1, seed, thresh, device)
    return out


def tissue_mask(W: int, H: int, seed: int = 4, background: float = 0.4, device="cuda",
                band: int = 1024) -> torch.Tensor:
    """(H, W) bool: the pixels he_slide draws as tissue (not background) --
    the ground truth of the region-of-interest task on these images."""
    thresh = background_threshold(W, H, seed, background, device)
    out = torch.empty((H, W), dtype=torch.bool, device=device)
    xs = torch.arange(W, device=device)
    for y0 in range(0, H, band):
        y1 = min(H, y0 + band)
        out[y0:y1] = _fbm(xs, torch.arange(y0, y1, device=device), 512, seed, 1) > thresh
    return out
