"""Small, independent Python restatements used to pin the oracle.

Each helper restates a definition straight from the paper (or from a textbook
closed form) in exact Python integers, without looking at how the oracle
computes it, so that a mistake in the oracle shows up as a disagreement.
"""
from __future__ import annotations

import numpy as np

# ring bit order shared with the C-ABI documentation: row-major 3x3 minus centre
RING = [(-1, -1), (0, -1), (1, -1), (-1, 0), (1, 0), (-1, 1), (0, 1), (1, 1)]
# circular order E, NE, N, NW, W, SW, S, SE (image y grows downwards)
_CIRC = [(1, 0), (1, -1), (0, -1), (-1, -1), (-1, 0), (-1, 1), (0, 1), (1, 1)]


def yokoi_simple(mask: int) -> bool:
    """4-connectivity Yokoi number C4 = sum over edge neighbours k of
    x_k - x_k x_{k+1} x_{k+2}; a point is (4,8)-simple iff C4 == 1."""
    f = {RING[i]: (mask >> i) & 1 for i in range(8)}
    x = [f[c] for c in _CIRC]
    c4 = sum(x[k] - x[k] * x[(k + 1) % 8] * x[(k + 2) % 8] for k in (0, 2, 4, 6))
    return c4 == 1


def stats(rgb: np.ndarray, labels: np.ndarray, K: int):
    """n, colour sums, coordinate sums per label (int64)."""
    H, W = labels.shape
    lab = labels.ravel().astype(np.int64)
    n = np.bincount(lab, minlength=K).astype(np.int64)
    S = np.stack([np.bincount(lab, weights=rgb[..., c].ravel().astype(np.float64), minlength=K)
                  for c in range(3)], 1).round().astype(np.int64)
    ys, xs = np.mgrid[0:H, 0:W]
    T = np.stack([np.bincount(lab, weights=xs.ravel().astype(np.float64), minlength=K),
                  np.bincount(lab, weights=ys.ravel().astype(np.float64), minlength=K)],
                 1).round().astype(np.int64)
    return n, S, T


def means(n, S, T, F: int):
    """Fixed-point means rounded half up: nearest integer to 2^F sum / n."""
    c = [[(2 ** (F + 1) * int(S[k, ch]) + int(n[k])) // (2 * int(n[k])) for ch in range(3)]
         for k in range(len(n))]
    mu = [[(2 ** (F + 1) * int(T[k, ax]) + int(n[k])) // (2 * int(n[k])) for ax in range(2)]
          for k in range(len(n))]
    return c, mu


def global_energy(rgb: np.ndarray, labels: np.ndarray, c, mu, p: dict) -> int:
    """Eq. (1) at pixel level with fixed-point means, exact integers:
    sum_p w_col |2^F I(p) - c|^2 + w_pos |2^F p - mu|^2
    + w_bnd 2^(2F) * #(unordered 4-adjacent pairs with different labels)."""
    F = p["frac_bits"]
    H, W = labels.shape
    e_col = 0
    e_pos = 0
    for y in range(H):
        for x in range(W):
            k = int(labels[y, x])
            for ch in range(3):
                d = (int(rgb[y, x, ch]) << F) - c[k][ch]
                e_col += d * d
            dx = (x << F) - mu[k][0]
            dy = (y << F) - mu[k][1]
            e_pos += dx * dx + dy * dy
    nb = int((labels[:, 1:] != labels[:, :-1]).sum() + (labels[1:, :] != labels[:-1, :]).sum())
    return p["w_col"] * e_col + p["w_pos"] * e_pos + p["w_bnd"] * (nb << (2 * F))


def components4(labels: np.ndarray) -> dict:
    """Number of 4-connected components of each label (plain BFS)."""
    H, W = labels.shape
    seen = np.zeros((H, W), bool)
    count: dict = {}
    for y0 in range(H):
        for x0 in range(W):
            if seen[y0, x0]:
                continue
            k = int(labels[y0, x0])
            count[k] = count.get(k, 0) + 1
            stack = [(y0, x0)]
            seen[y0, x0] = True
            while stack:
                y, x = stack.pop()
                for dy, dx in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                    yy, xx = y + dy, x + dx
                    if 0 <= yy < H and 0 <= xx < W and not seen[yy, xx] and labels[yy, xx] == k:
                        seen[yy, xx] = True
                        stack.append((yy, xx))
    return count


def components4_fast(labels: np.ndarray) -> dict:
    """Same as components4, via scipy.ndimage per label (large images)."""
    from scipy import ndimage
    out = {}
    objs = ndimage.find_objects(labels + 1)
    for k, sl in enumerate(objs):
        if sl is None:
            continue
        sub = labels[sl] == k
        _, nc = ndimage.label(sub, structure=[[0, 1, 0], [1, 1, 1], [0, 1, 0]])
        out[k] = nc
    return out
