"""Pins of the oracle's merge on underflow (Sec. 3.1, Eqs. (4)-(5)).

The merge energy is pinned to Eq. (1) itself: hand-derived values on a
three-cell image, and the pixel-level energy (tests/pyref.py, Python
integers) before and after relabelling on random label maps.  The pick and
conflict rules are pinned on a hand-traced case, and whole runs keep the
debug invariants (each pass's energies add up to the change of Eq. (1),
every label connected or empty, statistics equal to a recount).
"""
import numpy as np
import pytest

import oracle
from paper_1704_02083_amd import params, synth
from tests import pyref


def _three_cells():
    """12 x 4 image, three 4 x 4 cells: red, nearly red, blue."""
    rgb = np.zeros((4, 12, 3), np.uint8)
    rgb[:, 0:4] = (200, 0, 0)
    rgb[:, 4:8] = (190, 10, 0)
    rgb[:, 8:12] = (0, 0, 200)
    lab = np.repeat(np.repeat(np.arange(3, dtype=np.int32)[None, :], 4, 0), 4, 1)
    return rgb, lab


def _p(**kw):
    d = {"K": 0, "gx": 3, "gy": 1, "levels": [(1, [4])], "gate_level": -1, "frac_bits": 0,
         "max_sweeps": 16, "min_size": 8, "max_size": 40, "w_col": 1, "w_pos": 0, "w_bnd": 0,
         "merge": True}
    d.update(kw)
    return d


def test_merge_cost_hand_values():
    """Merging cell 1 into cell 0: the union mean is (195, 5, 0), so the
    colour term grows by 32 * (5^2 + 5^2) = 1600; into cell 2 the union mean
    is (95, 5, 100) and the term grows by 32 * 19050 = 609600.  With
    F = 0 the centroids round to x = 2, 6 and 4 (y = 2 throughout): the
    position term grows by 176 - 48 = 128, and the 4 shared pixel pairs stop
    being boundary: 1600 + 128 - 4 = 1724.  With F = 4 every mean is exact
    and each term scales by 2^8: 256 (1600 + 128 - 4) = 441344."""
    rgb, lab = _three_cells()
    assert oracle.merge_cost(rgb, _p(), lab, 3, 1, 0) == 1600
    assert oracle.merge_cost(rgb, _p(), lab, 3, 1, 2) == 609600
    full = _p(w_pos=1, w_bnd=1)
    assert oracle.merge_cost(rgb, full, lab, 3, 1, 0) == 1724
    assert oracle.merge_cost(rgb, full, lab, 3, 0, 1) == 1724      # symmetric
    assert oracle.merge_cost(rgb, dict(full, frac_bits=4), lab, 3, 1, 0) == 441344


@pytest.mark.parametrize("seed", range(6))
def test_merge_cost_is_eq1_difference(seed):
    """On random connected label maps the merge cost equals Eq. (1) at pixel
    level after relabelling m to k (means of the union) minus before."""
    rng = np.random.default_rng(100 + seed)
    W, H = int(rng.integers(6, 14)), int(rng.integers(6, 14))
    rgb = rng.integers(0, 256, size=(H, W, 3), dtype=np.uint8)
    gx, gy = 3, 2
    lab = oracle.init_labels(W, H, 1, gx, gy)
    K = gx * gy
    d = {"levels": [(1, [1])], "frac_bits": int(rng.integers(0, 5)),
         "w_col": int(rng.integers(0, 50)), "w_pos": int(rng.integers(0, 50)),
         "w_bnd": int(rng.integers(0, 5000))}
    F = d["frac_bits"]
    for m, k in ((0, 1), (1, 0), (0, 3), (4, 5), (2, 5)):
        n, S, T = pyref.stats(rgb, lab, K)
        c, mu = pyref.means(n, S, T, F)
        e0 = pyref.global_energy(rgb, lab, c, mu, d)
        lab2 = np.where(lab == m, k, lab).astype(np.int32)
        n2, S2, T2 = pyref.stats(rgb, lab2, K)
        n2 = [max(v, 1) for v in n2]      # the emptied label owns no pixel
        c2, mu2 = pyref.means(n2, S2, T2, F)
        e1 = pyref.global_energy(rgb, lab2, c2, mu2, d)
        full = dict(d, K=0, gx=gx, gy=gy, gate_level=-1, max_sweeps=1, min_size=0, max_size=1 << 20)
        assert oracle.merge_cost(rgb, full, lab, K, m, k) == e1 - e0, (m, k)


def test_merge_three_cells_traced():
    """Every cell is a single block that cannot leave without emptying its
    cell, so all three ask to merge.  Picks: 0 -> 1, 1 -> 0 (1600 < 609600),
    2 -> 1.  0 and 1 picked each other: the pair merges into label 0.  2's
    target leaves, so 2 waits; at the next quiet sweep it would reach 48 >
    max_size 40 pixels with label 0 and cannot merge."""
    rgb, _ = _three_cells()
    lab, st, rep = oracle.segment(rgb, _p(), debug=True)
    assert (lab[:, :8] == 0).all() and (lab[:, 8:] == 2).all()
    assert st[:, 0].tolist() == [32, 0, 16]
    assert st[1].tolist() == [0, 0, 0, 0, 0, 0]
    assert rep[0]["merges"] == 1 and rep[0]["converged"] == 1 and rep[0]["sweeps"] == 2
    # with room for it, 2 joins 0 at the next quiet sweep
    lab, st, rep = oracle.segment(rgb, _p(max_size=48), debug=True)
    assert (lab == 0).all() and rep[0]["merges"] == 2


def test_merge_off_changes_nothing():
    """merge = 0 is the plain method: identical output to a parameter set
    without the key."""
    img = synth.voronoi_blur(96, 64, regions=6, seed=3)
    p = params.default_params(96, 64, 12, levels=[(1, [8, 4, 2, 1])], min_size=100)
    a = oracle.segment(img, p)
    b = oracle.segment(img, dict(p, merge=False))
    assert (a[0] == b[0]).all() and a[2] == b[2]
    assert all(r["merges"] == 0 for r in a[2])


CASES = [
    # W, H, K, levels, min_size divisor, seed
    (128, 96, 24, [(1, [8, 4, 2, 1])], 4, 1),
    (160, 128, 40, params.THREE_LEVEL, 4, 2),
    (97, 61, 12, [(1, [8, 4, 2, 1])], 3, 3),
    (120, 80, 30, [(1, [4, 2, 1])], 2, 4),
]


@pytest.mark.parametrize("W,H,K,levels,div,seed", CASES)
def test_merge_runs_keep_invariants(W, H, K, levels, div, seed):
    """Debug runs with merges: per pass, the picked energies add up to the
    change of Eq. (1); every live label is 4-connected, merged labels are
    empty with zero sums; the live count drops by exactly the merges; no
    merge leaves a superpixel above max_size."""
    img = synth.voronoi_blur(W, H, regions=max(3, K // 2), seed=seed)
    p = params.default_params(W, H, K, levels=levels)
    A = (W * H) // oracle.n_superpixels(W, H, p)
    p.update(min_size=A // div, merge=True)
    lab, st, rep = oracle.segment(img, p, debug=True)
    Kp = oracle.n_superpixels(W, H, p)
    merges = sum(r["merges"] for r in rep)
    assert merges > 0
    live = st[:, 0] > 0
    assert int(live.sum()) == Kp - merges
    assert set(np.unique(lab).tolist()) == set(np.nonzero(live)[0].tolist())
    assert (st[~live] == 0).all()
    comps = pyref.components4_fast(lab)
    assert all(v == 1 for v in comps.values())
    n0 = np.bincount(oracle.init_labels(W, H, levels[0][0] * levels[0][1][0], *oracle.grid(W, H, K)).ravel(),
                     minlength=Kp)
    assert (st[live, 0] <= np.maximum(p["max_size"], n0[live])).all()
