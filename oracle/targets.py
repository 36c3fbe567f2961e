"""Reference for the gate's training target and for boundary recall
(test infrastructure only: the tests use it, the product never imports it).

Boundary recall (Sec. 4.2) counts the boundary pixels of a reference
segmentation that have a boundary pixel of the test segmentation close by.
A boundary pixel is one with a 4-neighbour (inside the image) of another
label; "close" is Chebyshev distance at most r.  A reference boundary pixel
without one is a miss; it is charged to the reference label and to the test
label of that pixel.  With the final plain labels as reference and the
labels at the gate point as test, a superpixel's charge says how far its
boundary still moves after the gate point.

Written pixel by pixel from that definition (slow; for small images).
"""
from __future__ import annotations

import numpy as np


def boundary_pixels(lab: np.ndarray) -> np.ndarray:
    """Boolean map: pixel has a 4-neighbour inside the image with another label."""
    H, W = lab.shape
    out = np.zeros((H, W), bool)
    for y in range(H):
        for x in range(W):
            v = lab[y, x]
            for dx, dy in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                u, w = x + dx, y + dy
                if 0 <= u < W and 0 <= w < H and lab[w, u] != v:
                    out[y, x] = True
                    break
    return out


def boundary_miss(ref: np.ndarray, test: np.ndarray, r: int, K: int):
    """Returns (miss per label (K,) int64, reference boundary pixels, misses)."""
    H, W = ref.shape
    bref, btest = boundary_pixels(ref), boundary_pixels(test)
    miss = np.zeros(K, np.int64)
    nb = nm = 0
    for y in range(H):
        for x in range(W):
            if not bref[y, x]:
                continue
            nb += 1
            win = btest[max(0, y - r):min(H, y + r + 1), max(0, x - r):min(W, x + r + 1)]
            if win.any():
                continue
            nm += 1
            for l in (ref[y, x], test[y, x]):
                if 0 <= l < K:
                    miss[l] += 1
    return miss, nb, nm
