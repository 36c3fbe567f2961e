"""Pins of the gate's reference code (features, network, Adam, targets)."""
import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_1704_02083_amd import params, synth


def test_bf16_round_to_nearest_even():
    cases = {1.0: 0x3F80, 1.0 + 2 ** -8: 0x3F80, 1.0 + 3 * 2 ** -8: 0x3F82,
             1.0 + 2 ** -9: 0x3F80, -2.5: 0xC020, 3.140625: 0x4049, 0.0: 0x0000}
    for v, bits in cases.items():
        assert int(mlp.to_bf16_bits(np.float32(v))) == bits, v
    x = np.random.default_rng(0).normal(size=1000).astype(np.float32)
    back = mlp.from_bf16_bits(mlp.to_bf16_bits(x))
    assert np.all(np.abs(back - x) <= np.abs(x) * 2 ** -8)


def test_backward_matches_central_differences():
    """fp64 gradient of the mean BCE equals central differences (rel 1e-6)."""
    rng = np.random.default_rng(1)
    theta = mlp.he_init(3)
    X = rng.normal(size=(37, 16))
    t = (rng.random(37) < 0.4).astype(np.float64)
    g, _ = mlp.grad(theta, X, t, bf16=False)
    h = 1e-6
    idx = np.concatenate([rng.choice(1024, 40, replace=False), 1024 + rng.choice(64, 10, replace=False),
                          1088 + rng.choice(4096, 60, replace=False), 5184 + rng.choice(64, 10, replace=False),
                          5248 + np.arange(64), [5312]])
    num = []
    for i in idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        num.append((mlp.loss(tp, X, t, bf16=False) - mlp.loss(tm, X, t, bf16=False)) / (2 * h))
    num = np.array(num)
    err = np.abs(num - g[idx])
    assert np.all(err <= 1e-6 * np.maximum(np.abs(num), 1e-3) + 1e-9), err.max()


def test_adam_first_step_closed_form():
    """From zero moments the first Adam step is -lr g / (|g| + eps)."""
    rng = np.random.default_rng(2)
    theta = rng.normal(size=100)
    g = rng.normal(size=100)
    new, m, v = mlp.adam_step(theta, np.zeros(100), np.zeros(100), g, 1, lr=1e-3)
    assert np.allclose(new - theta, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_logit_of_linear_network():
    """With W1 = [I;0] on 16 inputs, W2 = I, w3 = e_0 and zero biases, the
    network computes relu(x_0): a closed form for the forward pass."""
    parts = {"W1": np.zeros((64, 16)), "b1": np.zeros(64), "W2": np.eye(64), "b2": np.zeros(64),
             "w3": np.zeros(64), "b3": np.zeros(1)}
    parts["W1"][:16, :16] = np.eye(16)
    parts["w3"][0] = 1.0
    X = np.linspace(-2, 2, 32).reshape(2, 16)
    z, _ = mlp.forward(mlp.pack(parts), X, bf16=False)
    assert np.allclose(z, np.maximum(X[:, 0], 0))


def _two_region_features():
    """64 x 32 image, left half (30, 60, 90), right half (200, 100, 50),
    K = 2 (a 2 x 1 grid on the halves), one stage at B = 16."""
    img = np.zeros((32, 64, 3), np.uint8)
    img[:, :32] = (30, 60, 90)
    img[:, 32:] = (200, 100, 50)
    p = {"K": 2, "levels": [(1, [16])], "gate_level": -1, "frac_bits": 4, "max_sweeps": 8,
         "min_size": 0, "max_size": 1 << 30, "w_col": 1, "w_pos": 1, "w_bnd": 1}
    lab, st, rep, inv, mov = oracle.segment(img, p, track=True)
    return img, lab, st, mov, oracle.features(img, lab, 16, st, mov, 2, 1)


def test_features_two_regions_by_hand():
    img, lab, st, mov, f = _two_region_features()
    xs = np.mgrid[0:32, 0:64][1]
    assert (lab == (xs >= 32)).all()           # already optimal: nothing moves
    A = 64 * 32 // 2
    d = np.sqrt((170 ** 2 + 40 ** 2 + 40 ** 2) * 16 ** 2) / (255 * 16)
    exp0 = [30 / 255, 60 / 255, 90 / 255, 0, 0, 0, 1.0, 32 / (4 * np.sqrt(A)),
            32 ** 2 / (16 * A), 0.0, d, d, d, 0.0, 0.0, 1.0]
    exp1 = [200 / 255, 100 / 255, 50 / 255, 0, 0, 0, 1.0, 32 / (4 * np.sqrt(A)),
            32 ** 2 / (16 * A), 0.0, d, d, d, 0.0, 0.0, 1.0]
    assert np.allclose(f[0], exp0, rtol=1e-6, atol=1e-7)
    assert np.allclose(f[1], exp1, rtol=1e-6, atol=1e-7)


def test_features_std_and_drift():
    """Colour standard deviation from pixel second moments and the centroid
    drift, against numpy on a noisy image after refinement."""
    img = synth.voronoi_blur(96, 64, regions=8, seed=3)
    p = params.default_params(96, 64, 6, levels=[(1, [16, 8])])
    lab, st, rep, inv, mov = oracle.segment(img, p, track=True)
    gx, gy = oracle.grid(96, 64, 6)
    f = oracle.features(img, lab, 8, st, mov, gx, gy)
    A = 96 * 64 // 6
    ys, xs = np.mgrid[0:64, 0:96]
    for k in range(gx * gy):
        m = lab == k
        px = img[m].astype(np.float64)
        assert np.allclose(f[k, 3:6], px.std(0) / 64, rtol=1e-5, atol=1e-6)
        col, row = k % gx, k // gx
        cx0 = (2 * col + 1) * 96 / (2 * gx) - 0.5
        cy0 = (2 * row + 1) * 64 / (2 * gy) - 0.5
        drift = np.hypot(xs[m].mean() - cx0, ys[m].mean() - cy0) / np.sqrt(A)
        assert abs(f[k, 9] - drift) < 1e-6
        assert abs(f[k, 13] - mov[k] / m.sum()) < 1e-7


def test_gate_with_targets_is_plain():
    """Targets t (superpixels in any proposal past the gate level of the
    plain run) gate exactly the moves the plain run makes: by induction a
    gated-off superpixel never appears in a plain proposal, so the gated run
    with g = t reproduces the plain labels bit for bit."""
    img = synth.voronoi_blur(160, 128, regions=14, seed=8)
    img[:, :96] = (128, 128, 128)   # a flat region: its inner superpixels never move
    p = params.default_params(160, 128, 20, levels=params.THREE_LEVEL, gate_level=1)
    lab, st, rep, inv, mov = oracle.segment(img, p, track=True)
    assert 0 < inv.sum() < len(inv)
    gated = oracle.segment(img, p, gate=inv)
    assert (gated[0] == lab).all()
    # and every superpixel whose statistics changed after the gate is a target
    p1 = dict(p, levels=p["levels"][:1])
    _, st1, _ = oracle.segment(img, p1)
    changed = np.any(st1 != st, axis=1)
    assert np.all(inv[changed] == 1)


def _four_region_map():
    """40 x 20 label map worked by hand: 1 = x < 10, 2 = x >= 30, 0 = the
    middle columns above y = 10, 3 = the middle columns below.  Flat colours
    per label.  Superpixel 0 meets 1 along 10 pixel pairs (x = 9|10, y <
    10), 2 along 10 and 3 along 20 (y = 9|10); superpixel 3 likewise meets
    1 and 2 along 10 pairs each and 0 along 20."""
    H, W = 20, 40
    ys, xs = np.mgrid[0:H, 0:W]
    lab = np.where(xs < 10, 1, np.where(xs >= 30, 2, np.where(ys < 10, 0, 3))).astype(np.int32)
    col = {0: (100, 100, 100), 1: (0, 100, 100), 2: (100, 100, 160), 3: (100, 180, 100)}
    img = np.zeros((H, W, 3), np.uint8)
    for k, c in col.items():
        img[lab == k] = c
    st = np.zeros((4, 6), np.int64)
    for k in range(4):
        m = lab == k
        st[k] = [m.sum(), *(img[m].astype(np.int64).sum(0)), xs[m].sum(), ys[m].sum()]
    return img, lab, st


def test_features_contrast_max_rms_min_by_hand():
    """Features 10-12 (max, edge-weighted rms and min distance of the mean
    colours across the superpixel's boundary pixel pairs) on a map whose
    neighbour contrasts and shared edge lengths all differ, so that a max/min
    swap, an unweighted (per-neighbour) rms or a mean in place of the rms
    fails.  Means are fixed point with F = 4 (2^4 = 16 per colour unit), so a
    colour difference d gives a fixed-point distance 16 d and the features
    divide by 255 * 16 = 4080."""
    img, lab, st = _four_region_map()
    f = oracle.features(img, lab, 1, st, None, 2, 2)
    cs = 4080.0
    # superpixel 0 (100,100,100): to 1 d = 100 (10 pairs), to 2 d = 60 (10
    # pairs), to 3 d = 80 (20 pairs)
    d01, d02, d03 = 1600.0, 960.0, 1280.0
    rms0 = np.sqrt((10 * d01 ** 2 + 10 * d02 ** 2 + 20 * d03 ** 2) / 40)   # 1299.846...
    assert np.isclose(f[0, 10], d01 / cs, rtol=1e-6)
    assert np.isclose(f[0, 11], rms0 / cs, rtol=1e-6)
    assert np.isclose(f[0, 12], d02 / cs, rtol=1e-6)
    # the unweighted rms over the three neighbours (1306.4) and the mean
    # distance (1280) are both more than 1e-3 away
    assert abs(f[0, 11] - np.sqrt((d01 ** 2 + d02 ** 2 + d03 ** 2) / 3) / cs) > 1e-3
    assert abs(f[0, 11] - 1280.0 / cs) > 1e-3
    # superpixel 3 (100,180,100): to 1 |(100,80,0)| (10 pairs), to 2
    # |(0,80,60)| = 100 (10 pairs), to 0 80 (20 pairs)
    d31, d32, d30 = 16 * np.sqrt(100 ** 2 + 80 ** 2), 1600.0, 1280.0
    rms3 = np.sqrt((10 * d31 ** 2 + 10 * d32 ** 2 + 20 * d30 ** 2) / 40)
    assert np.isclose(f[3, 10], d31 / cs, rtol=1e-6)
    assert np.isclose(f[3, 11], rms3 / cs, rtol=1e-6)
    assert np.isclose(f[3, 12], d30 / cs, rtol=1e-6)
    # superpixel 1 (0,100,100): to 0 d = 100 (10 pairs), to 3 |(100,80,0)|
    # (10 pairs): max, rms and min of two equal-length edges
    d10, d13 = 1600.0, d31
    assert np.isclose(f[1, 10], d13 / cs, rtol=1e-6)
    assert np.isclose(f[1, 11], np.sqrt((d10 ** 2 + d13 ** 2) / 2) / cs, rtol=1e-6)
    assert np.isclose(f[1, 12], d10 / cs, rtol=1e-6)
    # boundary lengths (pixel pairs): 40, 20, 20, 40; A = 800 / 4 = 200
    for k, bl in enumerate([40, 20, 20, 40]):
        assert np.isclose(f[k, 7], bl / (4 * np.sqrt(200)), rtol=1e-6)
        assert np.isclose(f[k, 8], bl * bl / (16 * 200), rtol=1e-6)
    assert np.allclose(f[:, 3:6], 0) and np.allclose(f[:, 14], 0) and np.allclose(f[:, 15], 1)


def _stats_of(img, lab, K):
    """n, colour sums and coordinate sums per label, counted in numpy."""
    H, W, _ = img.shape
    ys, xs = np.mgrid[0:H, 0:W]
    st = np.zeros((K, 6), np.int64)
    for k in range(K):
        m = lab == k
        st[k] = [m.sum(), img[..., 0][m].sum(), img[..., 1][m].sum(), img[..., 2][m].sum(), xs[m].sum(), ys[m].sum()]
    return st


def test_roi_features_two_regions_by_hand():
    """The paper's four ROI features (Sec. 4) on a 4x4 image, left half label
    0 with rows alternating (10,20,30) / (14,20,30), right half label 1 of
    (100,100,100); F = 4, so the fixed-point means are (192,320,480) and
    (1600,1600,1600); four pixel pairs cross the border.  By hand:
    brightness 62/3 and 100; each side's neighbour brightness is the other's;
    the mean-colour distance is sqrt(1408^2 + 1280^2 + 1120^2) = 2208 fixed-
    point units; label 0's channel variances are 4, 0, 0."""
    img = np.zeros((4, 4, 3), np.uint8)
    img[:, :2] = (10, 20, 30)
    img[1::2, :2, 0] = 14
    img[:, 2:] = 100
    lab = np.zeros((4, 4), np.int32)
    lab[:, 2:] = 1
    f = oracle.roi_features(img, lab, _stats_of(img, lab, 2), 2, 1)
    want0 = [62 / 3 / 255, (62 / 3 - 100) / 255, 2208 / 4080, np.sqrt(4 / 3) / 64]
    want1 = [100 / 255, (100 - 62 / 3) / 255, 2208 / 4080, 0.0]
    assert np.allclose(f[0, :4], want0, rtol=1e-6, atol=1e-7)
    assert np.allclose(f[1, :4], want1, rtol=1e-6, atol=1e-7)
    assert (f[:, 4:15] == 0).all() and (f[:, 15] == 1).all()


def test_roi_features_edge_weighting_by_hand():
    """Three labels on a 4x3 image whose border pixel pairs are unequal:
        0 0 0 1
        0 0 0 1
        2 2 2 2
    label 0 (40,40,40) meets label 1 (100,100,100) on 2 pixel pairs and
    label 2 (mean (10,10,10), pixels alternating (8,10,12) / (12,10,8)) on 3;
    labels 1 and 2 meet on 1.  Neighbour brightness of label 0 is
    (2*100 + 3*10) / 5 = 46 (an unweighted mean would give 55, a size-
    weighted one 40), of label 1 (2*40 + 1*10) / 3 = 30, of label 2
    (3*40 + 1*100) / 4 = 55.  Label 0's rms distance is
    sqrt((2*3*960^2 + 3*3*480^2) / 5) fixed-point units; label 2's channel
    variances are 4, 0, 4."""
    img = np.zeros((3, 4, 3), np.uint8)
    img[:2, :3] = 40
    img[:2, 3] = 100
    img[2] = [(8, 10, 12), (12, 10, 8), (8, 10, 12), (12, 10, 8)]
    lab = np.array([[0, 0, 0, 1], [0, 0, 0, 1], [2, 2, 2, 2]], np.int32)
    f = oracle.roi_features(img, lab, _stats_of(img, lab, 3), 3, 1)
    assert np.allclose(f[:, 0], [40 / 255, 100 / 255, 10 / 255], rtol=1e-6)
    assert np.allclose(f[:, 1], [(40 - 46) / 255, (100 - 30) / 255, (10 - 55) / 255], rtol=1e-6, atol=1e-7)
    rms0 = np.sqrt((2 * 3 * 960 ** 2 + 3 * 3 * 480 ** 2) / 5)
    rms1 = np.sqrt((2 * 3 * 960 ** 2 + 1 * 3 * 1440 ** 2) / 3)
    rms2 = np.sqrt((3 * 3 * 480 ** 2 + 1 * 3 * 1440 ** 2) / 4)
    assert np.allclose(f[:, 2], np.array([rms0, rms1, rms2]) / 4080, rtol=1e-6)
    assert np.allclose(f[:, 3], [0, 0, np.sqrt(8 / 3) / 64], rtol=1e-6, atol=1e-7)


def test_roi_features_match_the_sixteen_on_shared_quantities():
    """On a refined H&E state, the ROI features that the learned gate's
    sixteen also measure agree with them: absolute brightness is the mean of
    features 0-2, extra-region dissimilarity is feature 11, intra-region
    dissimilarity is the quadratic mean of features 3-5 (same scales)."""
    img = synth.he_tile(192, 128, seed=17)
    p = params.default_params(192, 128, 24, levels=[(1, [16, 8, 4])])
    lab, st, _ = oracle.segment(img, p)
    gx, gy = oracle.grid(192, 128, 24)
    f16 = oracle.features(img, lab, 4, st, None, gx, gy)
    f4 = oracle.roi_features(img, lab, st, gx, gy)
    assert np.allclose(f4[:, 0], f16[:, :3].mean(1), rtol=1e-5, atol=1e-6)
    assert np.allclose(f4[:, 2], f16[:, 11], rtol=1e-5, atol=1e-6)
    assert np.allclose(f4[:, 3], np.sqrt((f16[:, 3:6].astype(np.float64) ** 2).mean(1)), rtol=1e-5, atol=1e-6)
