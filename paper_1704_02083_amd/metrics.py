"""Agreement of a segmentation with a reference segmentation.

The paper evaluates superpixels with boundary recall (BR) and
undersegmentation error (UE) (Sec. 4.2).  Here the reference is the plain
(ungated) result and the test is the gated one:

  boundary pixel  a pixel with a 4-neighbour of another label;
  BR              fraction of reference boundary pixels that have a test
                  boundary pixel within Chebyshev distance r (r = 2);
  UE              (1/N) sum over reference segments G of sum over test
                  segments S meeting G of min(|S & G|, |S \\ G|);
  disagreement    fraction of pixels whose labels differ (both runs start
                  from the same grid, so labels are comparable).
"""
from __future__ import annotations

import numpy as np


def boundary(labels: np.ndarray) -> np.ndarray:
    b = np.zeros(labels.shape, bool)
    dx = labels[:, 1:] != labels[:, :-1]
    dy = labels[1:, :] != labels[:-1, :]
    b[:, 1:] |= dx
    b[:, :-1] |= dx
    b[1:, :] |= dy
    b[:-1, :] |= dy
    return b


def _dilate(b: np.ndarray, r: int) -> np.ndarray:
    out = b.copy()
    H, W = b.shape
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            if dx == 0 and dy == 0:
                continue
            ys, yd = slice(max(0, dy), H + min(0, dy)), slice(max(0, -dy), H + min(0, -dy))
            xs, xd = slice(max(0, dx), W + min(0, dx)), slice(max(0, -dx), W + min(0, -dx))
            out[yd, xd] |= b[ys, xs]
    return out


def boundary_recall(ref: np.ndarray, test: np.ndarray, r: int = 2) -> float:
    br = boundary(ref)
    n = int(br.sum())
    if n == 0:
        return 1.0
    return float((_dilate(boundary(test), r) & br).sum()) / n


def undersegmentation_error(ref: np.ndarray, test: np.ndarray) -> float:
    ref = ref.ravel().astype(np.int64)
    test = test.ravel().astype(np.int64)
    N = ref.size
    nt = int(test.max()) + 1
    pair = ref * nt + test
    keys, counts = np.unique(pair, return_counts=True)
    s_of = keys % nt
    size_s = np.bincount(test, minlength=nt)
    err = np.minimum(counts, size_s[s_of] - counts).sum()
    return float(err) / N


def disagreement(ref: np.ndarray, test: np.ndarray) -> float:
    return float((ref != test).mean())


def agreement(ref: np.ndarray, test: np.ndarray) -> dict:
    return {"br": boundary_recall(ref, test), "ue": undersegmentation_error(ref, test),
            "disagreement": disagreement(ref, test)}
