"""The paper's own prediction step on the GPU: the four ROI features of
Sec. 4 (absolute and comparative brightness, extra- and intra-region
dissimilarity; gate_features "roi") feed the classifier of Eq. (6), and past
the gate level only pairs of superpixels of different predicted classes
refine (Eq. (7), rule "differ").  On every route that decides a gate (the
level-by-level state, one fused launch, a large image spread over a
cooperative launch, a slide's tiles) the features equal the oracle's within 1e-6, the
bits equal the oracle network's decision wherever its logit is 1e-2 clear
of the threshold, and the labels equal the oracle run under the GPU's bits;
a classifier trained on the four features finds the tissue."""
import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_1704_02083_amd import params, rapid, synth, synth_gpu

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0)
    yield c
    c.close()


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _roi_params(W, H, K, gate_level=1):
    p = params.default_params(W, H, K, levels=params.THREE_LEVEL, gate_level=gate_level)
    p["gate_rule"] = "differ"
    p["gate_features"] = "roi"
    return p


def _rand_model(seed):
    theta = mlp.he_init(seed).astype(np.float32)
    return theta, mlp.to_bf16_bits(theta).view(np.int16)


def _oracle_roi_features(img, p, gx, gy):
    """The oracle's ROI features at the gate point: the levels before the
    gate, then the four features on their labels."""
    p0 = dict(p, levels=p["levels"][:p["gate_level"]], gate_level=-1)
    lab0, s0, _ = oracle.segment(img, p0)
    return oracle.roi_features(img, lab0, s0, gx, gy)


def _check(img, p, X, g, labels, theta, thresh, gx, gy):
    Xo = _oracle_roi_features(img, p, gx, gy)
    diff = np.abs(X - Xo)
    assert diff.max() <= 1e-6 * max(1.0, float(np.abs(Xo).max())), diff.max()
    z, _ = mlp.forward(theta.astype(np.float64), Xo.astype(np.float64), bf16=True)
    clear = np.abs(z - thresh) > 1e-2
    assert (g[clear] == (z[clear] >= thresh)).all()
    ref, _, ref_rep = oracle.segment(img, p, gate=g)
    assert (labels == ref).all(), "%d labels differ" % int((labels != ref).sum())
    return ref_rep


def test_roi_features_state_route(ctx):
    """rapid_state_features with the ROI feature set after the first level
    equals the oracle's four features on the oracle's labels."""
    img = synth.he_tile(256, 192, seed=12)
    p = _roi_params(256, 192, 48)
    gx, gy = oracle.grid(256, 192, 48)
    st = ctx.state(_dev(img), p)
    st.refine_level(0)
    X = st.features().cpu().numpy()
    st.close()
    Xo = _oracle_roi_features(img, p, gx, gy)
    _say("case: roi features, state route, K=%d" % (gx * gy))
    assert np.abs(X - Xo).max() <= 1e-6
    assert (X[:, 4:15] == 0).all() and (X[:, 15] == 1).all()


@pytest.mark.parametrize("W,H,K,seed", [(256, 192, 48, 12), (300, 211, 60, 13)])
def test_roi_gate_fused_launch(ctx, W, H, K, seed):
    """One launch deciding the gate on the ROI features (rule differ):
    features, bits, labels and stage counters against the oracle, with the
    threshold at the median of the oracle's logits."""
    img = synth.he_tile(W, H, seed=seed)
    p = _roi_params(W, H, K)
    gx, gy = oracle.grid(W, H, K)
    theta, wb = _rand_model(seed)
    z, _ = mlp.forward(theta.astype(np.float64), _oracle_roi_features(img, p, gx, gy).astype(np.float64), bf16=True)
    thresh = float(np.median(z))
    _say("case: roi gate fused %dx%d K=%d thresh %.4f" % (W, H, K, thresh))
    labs, reps, X, g = ctx.segment_gated([_dev(img)], p, _dev(wb), thresh, features=True)
    g = g.cpu().numpy()
    assert 0 < g.sum() < len(g)
    ref_rep = _check(img, p, X.cpu().numpy(), g, labs[0].cpu().numpy(), theta, thresh, gx, gy)
    assert reps[0] == ref_rep
    # the caller-bits route of rapid_segment gives the same labels
    lab2, _ = ctx.segment(_dev(img), p, gate=_dev(g))
    assert (lab2.cpu().numpy() == labs[0].cpu().numpy()).all()


def test_roi_gate_large_image_cooperative(ctx):
    """A 1024^2 image spreads over the workgroups of one cooperative launch,
    which decides the gate point across the grid: the ROI features, bits and
    labels equal the oracle's and those of the same image on one workgroup."""
    import os
    img = synth.he_tile(1024, 1024, seed=33)
    p = _roi_params(1024, 1024, 4096)
    gx, gy = oracle.grid(1024, 1024, 4096)
    theta, wb = _rand_model(34)
    z, _ = mlp.forward(theta.astype(np.float64), _oracle_roi_features(img, p, gx, gy).astype(np.float64), bf16=True)
    thresh = float(np.median(z))
    _say("case: roi gate 1024^2 cooperative launch, thresh %.4f" % thresh)
    labs, _, X, g = ctx.segment_gated([_dev(img)], p, _dev(wb), thresh, features=True)
    g = g.cpu().numpy()
    _check(img, p, X.cpu().numpy(), g, labs[0].cpu().numpy(), theta, thresh, gx, gy)
    old = os.environ.get("RAPID_SHAPE")
    os.environ["RAPID_SHAPE"] = "1024,0,0"
    try:
        c1 = rapid.Context(0)
    finally:
        if old is None:
            os.environ.pop("RAPID_SHAPE", None)
        else:
            os.environ["RAPID_SHAPE"] = old
    try:
        labs1, _, X1, g1 = c1.segment_gated([_dev(img)], p, _dev(wb), thresh, features=True)
        assert (X1.cpu().numpy() == X.cpu().numpy()).all()
        assert (g1.cpu().numpy() == g).all()
        assert (labs1[0].cpu().numpy() == labs[0].cpu().numpy()).all()
    finally:
        c1.close()


def test_roi_gate_slide_tiles(ctx):
    """A ragged 1000 x 700 slide in 256-px tiles (64-px halo) gated on the
    ROI features inside one launch: every tile's features, bits and core
    labels against the oracle."""
    import torch
    W, H, T, h = 1000, 700, 256, 64
    rgb = synth_gpu.he_slide(W, H, seed=16, background=0.4, device="cuda", band=256)
    p = params.default_params(2048, 2048, 4096, levels=params.THREE_LEVEL, gate_level=1)
    p["gate_rule"], p["gate_features"] = "differ", "roi"
    theta, wb = _rand_model(35)
    lay = rapid.tile_layout(W, H, T, h, 32)
    img = rgb.cpu().numpy()

    def sub(t):
        ex0, ey0, ex1, ey1 = t["ext"]
        return np.ascontiguousarray(img[ey0:ey1, ex0:ex1])

    t0 = lay[0]
    z0, _ = mlp.forward(theta.astype(np.float64),
                        _oracle_roi_features(sub(t0), dict(p, K=0, gx=t0["gx"], gy=t0["gy"]), t0["gx"],
                                             t0["gy"]).astype(np.float64), bf16=True)
    thresh = float(np.median(z0))
    _say("case: roi gate slide %dx%d, thresh %.4f" % (W, H, thresh))
    labels, _, X, g = ctx.segment_slide(rgb, p, tile=T, halo=h, cell=32, w_bf16=torch.from_numpy(wb).cuda(),
                                        thresh=thresh, features=True)
    labels, X, g = labels.cpu().numpy(), X.cpu().numpy(), g.cpu().numpy()
    row = 0
    for ti, t in enumerate(lay):
        K = t["gx"] * t["gy"]
        s = sub(t)
        pt = dict(p, K=0, gx=t["gx"], gy=t["gy"])
        ex0, ey0, _, _ = t["ext"]
        cx0, cy0, cx1, cy1 = t["core"]
        Xo = _oracle_roi_features(s, pt, t["gx"], t["gy"])
        assert np.abs(X[row:row + K] - Xo).max() <= 1e-6
        z, _ = mlp.forward(theta.astype(np.float64), Xo.astype(np.float64), bf16=True)
        gt = g[row:row + K]
        clear = np.abs(z - thresh) > 1e-2
        assert (gt[clear] == (z[clear] >= thresh)).all()
        lab, _, _ = oracle.segment(s, pt, gate=gt)
        gid = (t["gid_y0"] + lab // t["gx"]) * t["gid_w"] + t["gid_x0"] + lab % t["gx"]
        exp = gid[cy0 - ey0:cy1 - ey0, cx0 - ex0:cx1 - ex0]
        assert (labels[cy0:cy1, cx0:cx1] == exp).all(), "tile %d" % ti
        row += K


def test_roi_classifier_on_the_four_features_finds_tissue(ctx):
    """The paper's pipeline end to end on the GPU: the classifier of Eq. (6)
    trained (balanced batches, as Sec. 4 samples half positive, half
    negative) on the four ROI features of 4 tiles for "most of the
    superpixel's pixels are tissue", then the gated run on a held-out tile:
    labels equal the oracle under the GPU's bits, and the ROI mask recovers
    the generator's tissue mask."""
    import torch
    from paper_1704_02083_amd import gate
    p = _roi_params(512, 512, 256)
    Xs, ts = [], []
    for i in range(4):
        rgb = synth_gpu.he_slide(512, 512, seed=600 + i, background=0.4, device="cuda")
        X, t = gate.roi_samples(ctx, rgb, synth_gpu.tissue_mask(512, 512, seed=600 + i, background=0.4), p)
        assert (X[:, 4:15] == 0).all()
        Xs.append(X)
        ts.append(t)
    _, w = gate.train(ctx, torch.cat(Xs), torch.cat(ts), epochs=20, batch=512, seed=0)
    rgb = synth_gpu.he_slide(512, 512, seed=699, background=0.4, device="cuda")
    labs, _, _, g = ctx.segment_gated([rgb], p, w, 0.0, report=False)
    _say("case: roi classifier on the four features, ROI superpixels %d of %d" % (int(g.sum().item()), g.numel()))
    ref, _, _ = oracle.segment(rgb.cpu().numpy(), p, gate=g.cpu().numpy())
    assert (labs[0].cpu().numpy() == ref).all()
    sc = gate.roi_scores(gate.roi_mask(labs[0], g), synth_gpu.tissue_mask(512, 512, seed=699, background=0.4))
    _say("ROI %s" % sc)
    assert sc["f1"] >= 0.9
