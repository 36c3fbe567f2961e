"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these re-types the oracle's own formulas: each compares it with a
closed form, a textbook routine, a hand-derived special case or an
independent exact-integer restatement (tests/pyref.py).
"""
import numpy as np
import pytest

import oracle
from paper_1704_02083_amd import params, synth
from tests import pyref


# ------------------------------------------------------------------ topology

def test_simple_point_matches_yokoi_number():
    """Topology term of Eq. (1): the oracle's flood-fill (4,8) simple-point
    test equals the Yokoi 4-connectivity number C4 == 1 on all 256 rings."""
    for m in range(256):
        assert oracle.simple(m) == pyref.yokoi_simple(m), m


def test_simple_point_count():
    """116 of the 256 ring masks are simple; the only mask with one
    foreground component but a non-simple centre is the full ring."""
    assert sum(oracle.simple(m) for m in range(256)) == 116
    assert not oracle.simple(255)
    assert not oracle.simple(0)        # isolated block: removal deletes the label


def test_simple_point_removal_keeps_connectivity():
    """Property: whenever the local test accepts removing a block from label
    a, the rest of a stays 4-connected (global BFS), on random labellings."""
    rng = np.random.default_rng(7)
    checked = 0
    for trial in range(200):
        # a random 4-connected set grown from one seed cell
        lab = np.zeros((7, 7), np.int32)
        y, x = rng.integers(0, 7, size=2)
        lab[y, x] = 1
        for _ in range(int(rng.integers(3, 30))):
            ys, xs = np.nonzero(lab == 1)
            i = int(rng.integers(0, len(ys)))
            dy, dx = ((1, 0), (-1, 0), (0, 1), (0, -1))[int(rng.integers(0, 4))]
            yy, xx = ys[i] + dy, xs[i] + dx
            if 0 <= yy < 7 and 0 <= xx < 7:
                lab[yy, xx] = 1
        assert pyref.components4(lab).get(1, 0) == 1
        for y in range(7):
            for x in range(7):
                if lab[y, x] != 1:
                    continue
                mask = 0
                for r, (dx, dy) in enumerate(pyref.RING):
                    xx, yy = x + dx, y + dy
                    if 0 <= xx < 7 and 0 <= yy < 7 and lab[yy, xx] == 1:
                        mask |= 1 << r
                if oracle.simple(mask):
                    l2 = lab.copy()
                    l2[y, x] = 2
                    c = pyref.components4(l2)
                    assert c.get(1, 0) == 1
                    checked += 1
    assert checked > 100


# ---------------------------------------------------------------------- grid

@pytest.mark.parametrize("W,H,K,exp", [(256, 256, 64, (8, 8)), (481, 321, 400, (25, 16)),
                                       (321, 481, 400, (17, 24)), (4096, 4096, 16384, (128, 128)),
                                       (64, 64, 4, (2, 2)), (100, 10, 10, (10, 1))])
def test_grid_shape(W, H, K, exp):
    assert oracle.grid(W, H, K) == exp


def test_grid_aligned_cells():
    """For a 256x256 image and 8x8 cells the block-centre rule reduces to the
    regular 32-px grid (Algorithm RAPID, grid initialisation)."""
    lab = oracle.init_labels(256, 256, 16, 8, 8)
    ys, xs = np.mgrid[0:256, 0:256]
    assert (lab == (ys // 32) * 8 + xs // 32).all()


@pytest.mark.parametrize("W,H,K,B0", [(481, 321, 400, 16), (321, 481, 400, 16), (97, 61, 12, 8),
                                      (33, 17, 2, 16)])
def test_grid_onto_and_connected(W, H, K, B0):
    """Every initial superpixel is non-empty, a union of whole blocks and
    4-connected, even with ragged edge blocks."""
    gx, gy = oracle.grid(W, H, K)
    lab = oracle.init_labels(W, H, B0, gx, gy)
    assert set(np.unique(lab)) == set(range(gx * gy))
    comps = pyref.components4_fast(lab)
    assert all(v == 1 for v in comps.values())
    # constant on blocks
    for y in range(0, H, B0):
        for x in range(0, W, B0):
            blk = lab[y:y + B0, x:x + B0]
            assert (blk == blk[0, 0]).all()


# ------------------------------------------------------------- special cases

def _edge_params(**kw):
    d = {"K": 2, "levels": [(1, [16, 8, 4, 2, 1])], "gate_level": -1,
         "frac_bits": 4, "max_sweeps": 64, "min_size": 0, "max_size": 1 << 40,
         "w_col": 1, "w_pos": 0, "w_bnd": 0}
    d.update(kw)
    return d


def test_edge_snapping_vertical():
    """Worked by hand: a 64x64 image with columns x < 37 at grey 50 and
    x >= 37 at grey 200, two superpixels (32-px wide halves), colour term
    only, no size limits.  Stage 16 keeps the mixed block [32,48) right
    (cost 1.38M < 3.96M per 16 rows); stage 8 moves [32,40) left (540k <
    654k per 8 rows); stage 4 moves [36,40) back right (90k < 231k);
    stage 2 keeps [36,38) right (41.9k < 45k); stage 1 moves column 36 left.
    The boundary ends exactly on the step, between x = 36 and x = 37."""
    img = np.zeros((64, 64, 3), np.uint8)
    img[:, :37] = 50
    img[:, 37:] = 200
    lab, st, rep = oracle.segment(img, _edge_params(), debug=True)
    xs = np.mgrid[0:64, 0:64][1]
    assert (lab == (xs >= 37)).all()


def test_edge_snapping_horizontal():
    """The same step transposed and mirrored (rows y < 27 at 200, y >= 27 at
    50, explicit 1x2 grid): the boundary moves from y = 32 to y = 27."""
    img = np.zeros((64, 64, 3), np.uint8)
    img[27:] = 50
    img[:27] = 200
    lab, st, rep = oracle.segment(img, _edge_params(K=0, gx=1, gy=2), debug=True)
    ys = np.mgrid[0:64, 0:64][0]
    assert (lab == (ys >= 27)).all()


def test_equal_means_do_not_trade():
    """Strict improvement: two superpixels of identical flat colour and no
    position or boundary term never exchange a block."""
    img = np.full((64, 64, 3), 77, np.uint8)
    lab, st, rep = oracle.segment(img, _edge_params(), debug=True)
    assert sum(r["proposals"] for r in rep) == 0
    xs = np.mgrid[0:64, 0:64][1]
    assert (lab == (xs >= 32)).all()


def test_flat_mosaic_no_proposals():
    """A flat grid-aligned mosaic with distinct colours is already optimal:
    no block has a better label, so nothing is proposed."""
    img = synth.flat_mosaic(128, 128, 32, seed=3)
    p = params.default_params(128, 128, 16)
    lab, st, rep = oracle.segment(img, p)
    assert sum(r["proposals"] for r in rep) == 0
    ys, xs = np.mgrid[0:128, 0:128]
    assert (lab == (ys // 32) * 4 + xs // 32).all()


def test_single_superpixel_has_no_boundary():
    img = synth.voronoi_blur(64, 64, regions=5, seed=2)
    p = params.default_params(64, 64, 1)
    lab, st, rep = oracle.segment(img, p)
    assert (lab == 0).all()
    assert all(r["active"] == 0 for r in rep)


def test_colour_only_moves_go_to_nearest_mean():
    """With w_pos = w_bnd = 0 the energy of a block is its colour SSE, so
    every proposal picks the admissible neighbour label whose mean colour is
    nearest to the block (exact integer check on every class of a state)."""
    img = synth.voronoi_blur(48, 48, regions=6, seed=5)
    p = {"K": 9, "levels": [(1, [4, 2, 1])], "gate_level": -1, "frac_bits": 4,
         "max_sweeps": 64, "min_size": 0, "max_size": 1 << 40, "w_col": 3, "w_pos": 0, "w_bnd": 0}
    gx, gy = oracle.grid(48, 48, 9)
    lab = oracle.init_labels(48, 48, 4, gx, gy)
    n, S, T = pyref.stats(img, lab, 9)
    c, _ = pyref.means(n, S, T, 4)
    total = 0
    for cls in range(9):
        props, de = oracle.propose_class(img, p, lab, 9, 4, cls)
        for (b, a, k) in props:
            bx, by = b % 12, b // 12
            blk = img[by * 4:by * 4 + 4, bx * 4:bx * 4 + 4].reshape(-1, 3).astype(np.int64) << 4

            def sse(q):
                return int(((blk - np.array(c[q])) ** 2).sum())
            nbrs = {lab[by * 4, bx * 4 - 4] if bx > 0 else -1, lab[by * 4, bx * 4 + 4] if bx < 11 else -1,
                    lab[by * 4 - 4, bx * 4] if by > 0 else -1, lab[by * 4 + 4, bx * 4] if by < 11 else -1}
            nbrs.discard(-1)
            nbrs.discard(a)
            best = min(sorted(nbrs), key=sse)
            assert k == best and sse(k) < sse(a)
            total += 1
    assert total > 0


# --------------------------------------------------------- Eq. (8) transform

def test_eq8_centroid_transform_zero_based():
    """Eq. (8) maps a centroid from a level with ratio C to the next finer
    one.  With 0-based pixel indices the offset is +(C-1)/2 (the paper's
    minus sign holds for 1-based indices); in sums: T_f = C^3 T_c +
    C^2 (C-1)/2 n_c and n_f = C^2 n_c.  Checked on random coarse labels."""
    rng = np.random.default_rng(11)
    for C in (2, 4, 5):
        lc = rng.integers(0, 6, size=(9, 7))
        lf = np.kron(lc, np.ones((C, C), np.int64))
        for k in range(6):
            yc, xc = np.nonzero(lc == k)
            yf, xf = np.nonzero(lf == k)
            if len(xc) == 0:
                continue
            assert len(xf) == C * C * len(xc)
            assert xf.sum() == C ** 3 * xc.sum() + C * C * (C - 1) // 2 * len(xc) if C % 2 else True
            assert 2 * xf.sum() == 2 * C ** 3 * xc.sum() + C * C * (C - 1) * len(xc)
            assert 2 * yf.sum() == 2 * C ** 3 * yc.sum() + C * C * (C - 1) * len(yc)
            # the mean itself: mu_f = C mu_c + (C - 1)/2
            assert abs(xf.mean() - (C * xc.mean() + (C - 1) / 2)) < 1e-9
            # 1-based indices: mu_f' = C mu_c' - (C - 1)/2 as printed
            assert abs((xf + 1).mean() - (C * (xc + 1).mean() - (C - 1) / 2)) < 1e-9


def test_three_levels_equal_single_level():
    """Levels are exact box sums, so three levels of ratio 4 with blocks
    1 | 2,1 | 2,1 (effective 16 | 8,4 | 2,1) equal one level 16,8,4,2,1."""
    img = synth.voronoi_blur(128, 96, regions=10, seed=9)
    p1 = params.default_params(128, 96, 24)
    p3 = params.default_params(128, 96, 24, levels=params.THREE_LEVEL)
    l1, s1, r1 = oracle.segment(img, p1)
    l3, s3, r3 = oracle.segment(img, p3)
    assert (l1 == l3).all() and (s1 == s3).all()
    strip = [{k: v for k, v in r.items() if k != "level"} for r in r1]
    assert strip == [{k: v for k, v in r.items() if k != "level"} for r in r3]


# ----------------------------------------------------------------- invariants

def _check_final(img, p, lab, st, K):
    comps = pyref.components4_fast(lab)
    assert len(comps) == K and all(v == 1 for v in comps.values())
    n, S, T = pyref.stats(img, lab, K)
    assert (st[:, 0] == n).all() and (st[:, 1:4] == S).all() and (st[:, 4:6] == T).all()


def test_config1_invariants_and_energy():
    """Config 1 under the oracle's per-class debug checks (energy identity
    and monotonicity, recount, connectivity), then independent checks of the
    result and of the energy drop with tests/pyref.py."""
    img = synth.voronoi_blur()
    p = params.config1()
    lab, st, rep = oracle.segment(img, p, debug=True)
    _check_final(img, p, lab, st, 64)
    lab0 = oracle.init_labels(256, 256, 16, 8, 8)
    for L in (lab0, lab):
        n, S, T = pyref.stats(img, L, 64)
    n0, S0, T0 = pyref.stats(img, lab0, 64)
    c0, m0 = pyref.means(n0, S0, T0, 4)
    n1, S1, T1 = pyref.stats(img, lab, 64)
    c1, m1 = pyref.means(n1, S1, T1, 4)
    e0 = pyref.global_energy(img, lab0, c0, m0, p)
    e1 = pyref.global_energy(img, lab, c1, m1, p)
    assert e1 < e0
    # size bounds: undersized cannot shrink, oversized cannot grow
    assert (n1 >= np.minimum(p["min_size"], n0)).all()
    assert (n1 <= np.maximum(p["max_size"], n0)).all()
    assert all(r["converged"] for r in rep)


@pytest.mark.parametrize("seed,shape", [(1000, (481, 321)), (1100, (321, 481))])
def test_config2_invariants(seed, shape):
    W, H = shape
    img = synth.voronoi_gradient(W, H, seed=seed)
    p = params.config2(W, H)
    lab, st, rep = oracle.segment(img, p, debug=False)
    K = oracle.n_superpixels(W, H, p)
    _check_final(img, p, lab, st, K)


@pytest.mark.parametrize("seed", [21, 22, 23])
def test_random_small_debug(seed):
    rng = np.random.default_rng(seed)
    W, H = int(rng.integers(20, 70)), int(rng.integers(20, 70))
    img = synth.voronoi_blur(W, H, regions=int(rng.integers(3, 12)), seed=seed)
    K = int(rng.integers(2, 12))
    p = params.default_params(W, H, K, levels=[(1, [4, 2, 1])], min_size=int(rng.integers(0, 40)))
    p["w_pos"] = int(rng.integers(0, 300))
    p["w_bnd"] = int(rng.integers(0, 5000))
    try:
        lab, st, rep = oracle.segment(img, p, debug=True)
    except RuntimeError:
        pytest.skip("grid does not fit")
    _check_final(img, p, lab, st, oracle.n_superpixels(W, H, p))


def test_order_independence():
    """Within a class every proposal reads the class-start state and the
    updates are integer sums, so any processing order gives the same result."""
    img = synth.voronoi_blur(96, 80, regions=9, seed=4)
    p = params.default_params(96, 80, 20)
    base = oracle.segment(img, p)
    for s in (1, 2, 3):
        other = oracle.segment(img, p, shuffle_seed=s)
        assert (other[0] == base[0]).all() and (other[1] == base[1]).all()
        assert other[2] == base[2]


# ------------------------------------------------------------------- the gate

def test_gate_all_ones_is_plain():
    """pair-active(a, k) = g_a or g_k: a gate that marks every superpixel
    leaves the plain method unchanged (Eq. (7) reduces to Eq. (2))."""
    img = synth.voronoi_blur(128, 128, regions=12, seed=6)
    p = params.default_params(128, 128, 16, levels=params.THREE_LEVEL, gate_level=1)
    plain = oracle.segment(img, p)
    K = oracle.n_superpixels(128, 128, p)
    gated = oracle.segment(img, p, gate=np.ones(K, np.uint8))
    assert (plain[0] == gated[0]).all() and plain[2] == gated[2]


def test_gate_all_zero_freezes_after_gate_level():
    """With no superpixel marked, no pair is active past the gate level:
    the labels after level 1 are final."""
    img = synth.voronoi_blur(128, 128, regions=12, seed=6)
    p = params.default_params(128, 128, 16, levels=params.THREE_LEVEL, gate_level=1)
    K = oracle.n_superpixels(128, 128, p)
    gated = oracle.segment(img, p, gate=np.zeros(K, np.uint8))
    p1 = dict(p, levels=p["levels"][:1], gate_level=-1)
    lvl1 = oracle.segment(img, p1)
    assert (gated[0] == lvl1[0]).all()
    assert all(r["proposals"] == 0 and r["active"] == 0 for r in gated[2][1:])


def _gate_case():
    img = synth.voronoi_blur(128, 128, regions=12, seed=6)
    p = params.default_params(128, 128, 16, levels=params.THREE_LEVEL, gate_level=1)
    K = oracle.n_superpixels(128, 128, p)
    lvl1 = oracle.segment(img, dict(p, levels=p["levels"][:1], gate_level=-1))
    return img, p, K, lvl1


def test_gate_rule_both_all_ones_is_plain():
    img, p, K, _ = _gate_case()
    plain = oracle.segment(img, p)
    gated = oracle.segment(img, dict(p, gate_rule="both"), gate=np.ones(K, np.uint8))
    assert (plain[0] == gated[0]).all() and plain[2] == gated[2]


def test_gate_rule_differ_one_class_freezes():
    """Pairs refine only across a class border: one class everywhere means
    no pair is active past the gate level."""
    img, p, K, lvl1 = _gate_case()
    for v in (0, 1):
        gated = oracle.segment(img, dict(p, gate_rule="differ"), gate=np.full(K, v, np.uint8))
        assert (gated[0] == lvl1[0]).all()
        assert all(r["active"] == 0 for r in gated[2][1:])


def test_gate_rule_both_freezes_unmarked_superpixels():
    """Under the rule "both" a superpixel the gate leaves unmarked takes
    part in no pair, so it keeps exactly the pixels it had at the gate
    point, while marked ones still move."""
    img, p, K, lvl1 = _gate_case()
    g = (np.random.default_rng(3).random(K) < 0.5).astype(np.uint8)
    lab = oracle.segment(img, dict(p, gate_rule="both"), gate=g)[0]
    for k in range(K):
        if not g[k]:
            assert ((lab == k) == (lvl1[0] == k)).all(), k
    assert (lab != lvl1[0]).any()


def test_gate_rule_differ_moves_only_across_classes():
    """Under the rule "differ" with two classes that split the image into
    halves, every pixel that changes label past the gate point lies near the
    class border (a move needs a neighbour of the other class)."""
    img, p, K, lvl1 = _gate_case()
    gx, gy = oracle.grid(128, 128, 16)
    g = np.array([1 if (k % gx) >= gx // 2 else 0 for k in range(K)], np.uint8)
    lab = oracle.segment(img, dict(p, gate_rule="differ"), gate=g)[0]
    # a superpixel not adjacent to the other class at the gate point and
    # whose neighbours are all of its own class cannot change
    changed = lab != lvl1[0]
    assert changed.any()
    cls_before = g[lvl1[0]]
    cls_after = g[lab]
    # pixels keep their class unless they sit in a superpixel that touched
    # the border; the class map changes only in the columns around it
    xs = np.nonzero((cls_before != cls_after).any(axis=0))[0]
    border = 128 * (gx // 2) // gx
    assert xs.size and xs.min() >= border - 48 and xs.max() < border + 48


# --------------------------------------------------------- class size filter

def _filter_case(min_size, max_size):
    """8x4 image, two superpixels (x < 4 left, x >= 4 right), column x = 3
    white on a black left half: every pixel of column 3 prefers the right
    label.  Block size 1, colour term only.  Column-3 pixels fall in class 0
    (rows 0 and 3), class 3 (row 1) and class 6 (row 2)."""
    img = np.zeros((4, 8, 3), np.uint8)
    img[:, 3:] = 255
    p = {"K": 0, "gx": 2, "gy": 1, "levels": [(1, [1])], "gate_level": -1, "frac_bits": 4,
         "max_sweeps": 64, "min_size": min_size, "max_size": max_size,
         "w_col": 1, "w_pos": 0, "w_bnd": 0}
    lab, st, rep = oracle.segment(img, p, debug=True)
    return lab[:, 3].tolist(), rep[0]


def test_filter_upper_bound_reached_exactly():
    """max = 18: class 0 moves rows 0 and 3 (16 + 2 = 18 is allowed), then
    rows 1 and 2 are dropped (18 + 1 > 18)."""
    col, rep = _filter_case(0, 18)
    assert col == [1, 0, 0, 1] and rep["commits"] == 2


def test_filter_upper_bound_rejects_class_aggregate():
    """max = 17: each class-0 proposal fits alone (16 + 1) but together they
    would give 18, so both are rejected; class 3 then moves row 1 alone and
    everything else is dropped."""
    col, rep = _filter_case(0, 17)
    assert col == [0, 1, 0, 0] and rep["commits"] == 1 and rep["proposals"] == 3


def test_frontier_reactivation_count():
    """After a sweep only eligible blocks within one block of a changed block
    stay active.  In the max = 17 case sweep 1 visits the 8 eligible blocks
    of columns 3 and 4; only (3, 1) changes; sweep 2 visits the eligible
    blocks of x in [2, 4], y in [0, 2]: (2,1), (3,0), (3,1), (3,2), (4,0),
    (4,2) -- 6, not the 8 eligible blocks of the whole image -- and commits
    nothing, so the stage ends after 2 sweeps with 8 + 6 block visits."""
    col, rep = _filter_case(0, 17)
    assert rep["sweeps"] == 2 and rep["converged"] == 1
    assert rep["active"] == 8 + 6


def test_filter_lower_bound_reached_exactly():
    """min = 14: class 0 takes the left from 16 to 14 (allowed); row 1 and
    row 2 are then skipped (14 - 1 < 14)."""
    col, rep = _filter_case(14, 1 << 40)
    assert col == [1, 0, 0, 1] and rep["commits"] == 2 and rep["skip_min"] > 0


def test_filter_lower_bound_rejects_class_aggregate():
    """min = 15: the two class-0 moves together would leave 14 < 15, so both
    are rejected; class 3 moves row 1 (16 - 1 = 15) and the rest is skipped."""
    col, rep = _filter_case(15, 1 << 40)
    assert col == [0, 1, 0, 0] and rep["commits"] == 1 and rep["proposals"] == 3


def test_sweep_cap_reports_not_converged():
    """max_sweeps = 1: every stage runs exactly one sweep and reports
    converged only when that sweep committed nothing."""
    img = synth.voronoi_blur(128, 96, regions=10, seed=5)
    p = params.default_params(128, 96, 24, max_sweeps=1)
    _, _, rep = oracle.segment(img, p, debug=True)
    assert all(r["sweeps"] == 1 for r in rep)
    assert all(r["converged"] == (1 if r["commits"] == 0 else 0) for r in rep)
    assert any(r["converged"] == 0 for r in rep)


@pytest.mark.parametrize("seed", range(3))
def test_energy_equals_pixel_level_eq1(seed):
    """orc_energy is Eq. (1) at pixel level with fixed-point means: equal,
    as an exact integer, to the restatement in Python integers, on a
    refined state and on a random (disconnected) label map, with random
    weights and F."""
    rng = np.random.default_rng(50 + seed)
    W, H = 23 + 5 * seed, 17 + 3 * seed
    img = rng.integers(0, 256, size=(H, W, 3), dtype=np.uint8)
    p = dict(params.default_params(W, H, 6, levels=[(1, [4, 2, 1])]),
             w_col=int(rng.integers(1, 50)), w_pos=int(rng.integers(0, 50)), w_bnd=int(rng.integers(0, 5000)),
             frac_bits=int(rng.integers(0, 5)), min_size=0)
    K = oracle.n_superpixels(W, H, p)
    refined, _, _ = oracle.segment(img, p)
    rand = rng.integers(0, K, size=(H, W)).astype(np.int32)
    rand.ravel()[:K] = np.arange(K)   # every label non-empty
    for lab in (refined, rand):
        n, S, T = pyref.stats(img, lab, K)
        c, mu = pyref.means(n, S, T, p["frac_bits"])
        assert oracle.energy(img, p, lab) == pyref.global_energy(img, lab, c, mu, p)
