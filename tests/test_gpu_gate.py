"""GPU parity of the gate: features, targets, network forward/backward,
Adam, and gated segmentation against the CPU references."""
import numpy as np
import pytest

import oracle
from oracle import mlp, targets
from paper_1704_02083_amd import params, synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0)
    yield c
    c.close()


def _dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _he_case():
    img = synth.he_tile(256, 192, seed=12)
    p = params.default_params(256, 192, 48, levels=params.THREE_LEVEL, gate_level=1)
    return img, p


def test_features_and_targets_match_oracle(ctx):
    import torch
    img, p = _he_case()
    gx, gy = oracle.grid(256, 192, 48)
    K = gx * gy
    _say("case: features 256x192 H&E K=%d" % K)
    st = ctx.state(_dev(img), p)
    moved = torch.zeros(K, dtype=torch.int64, device="cuda")
    involved = torch.zeros(K, dtype=torch.uint8, device="cuda")
    st.track(None, moved)
    st.refine_level(0)
    X = st.features().cpu().numpy()
    moved0 = moved.cpu().numpy().copy()
    # oracle: level 0 only
    p0 = dict(p, levels=p["levels"][:1], gate_level=-1)
    lab0, s0, _, _, mov0 = oracle.segment(img, p0, track=True)
    Xo = oracle.features(img, lab0, 16, s0, mov0, gx, gy)
    assert (moved0 == mov0).all()
    diff = np.abs(X - Xo)
    assert diff.max() <= 1e-6 * max(1.0, np.abs(Xo).max()), diff.max()
    # targets: involvement after the gate level
    st.track(involved, moved)
    st.refine_level(1)
    st.refine_level(2)
    lab, _ = st.export()
    _, _, _, inv, mov = oracle.segment(img, p, track=True)
    assert (involved.cpu().numpy() == inv).all()
    assert (moved.cpu().numpy() == mov).all()
    st.close()


def _rand_model(seed):
    theta = mlp.he_init(seed).astype(np.float32)
    return theta, mlp.to_bf16_bits(theta).view(np.int16)


def test_mlp_forward_matches_oracle(ctx):
    import torch
    rng = np.random.default_rng(5)
    N = 1000   # not a multiple of 16
    X = rng.normal(size=(N, 16)).astype(np.float32)
    theta, wb = _rand_model(7)
    logits, gate = ctx.mlp_forward(_dev(X), _dev(wb), 0.25)
    logits = logits.cpu().numpy()
    ref, _ = mlp.forward(theta.astype(np.float64), X.astype(np.float64), bf16=True)
    err = np.abs(logits - ref)
    _say("mlp forward max abs err %.3g" % err.max())
    assert err.max() <= 1e-2
    far = np.abs(ref - 0.25) > 1e-2
    assert (gate.cpu().numpy()[far] == (ref[far] >= 0.25)).all()


def test_mlp_grad_matches_oracle(ctx):
    rng = np.random.default_rng(6)
    N = 2000
    X = (rng.normal(size=(N, 16)) * 0.7).astype(np.float32)
    t = (rng.random(N) < 0.45).astype(np.uint8)
    idx = rng.choice(N, 777, replace=False).astype(np.int32)
    theta, wb = _rand_model(9)
    g, logits = ctx.mlp_grad(_dev(X), _dev(t), _dev(idx), _dev(wb))
    g = g.cpu().numpy().astype(np.float64)
    gr, zr = mlp.grad(theta.astype(np.float64), X[idx].astype(np.float64), t[idx].astype(np.float64),
                      bf16=True)
    assert np.abs(logits.cpu().numpy() - zr).max() <= 1e-2
    parts_g, parts_r = mlp.unpack(g), mlp.unpack(gr)
    for name, _ in mlp.SIZES:
        a, b = parts_g[name].ravel(), parts_r[name].ravel()
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-12)
        _say("grad %s rel L2 %.3g" % (name, rel))
        assert rel <= 2 ** -6, name


def test_mlp_grad_deterministic(ctx):
    rng = np.random.default_rng(11)
    X = rng.normal(size=(5000, 16)).astype(np.float32)
    t = (rng.random(5000) < 0.5).astype(np.uint8)
    idx = np.arange(4096, dtype=np.int32)
    theta, wb = _rand_model(3)
    g1, _ = ctx.mlp_grad(_dev(X), _dev(t), _dev(idx), _dev(wb))
    g2, _ = ctx.mlp_grad(_dev(X), _dev(t), _dev(idx), _dev(wb))
    assert (g1.cpu().numpy() == g2.cpu().numpy()).all()


def test_adam_first_step(ctx):
    """One epoch of one balanced batch (all 512 samples): the update equals
    the closed-form first Adam step -lr g / (|g| + eps)."""
    import torch
    rng = np.random.default_rng(12)
    X = rng.normal(size=(512, 16)).astype(np.float32)
    t = np.zeros(512, np.uint8)
    t[rng.choice(512, 256, replace=False)] = 1
    theta, wb = _rand_model(4)
    g, _ = ctx.mlp_grad(_dev(X), _dev(t), _dev(np.arange(512, dtype=np.int32)), _dev(wb))
    g = g.cpu().numpy()
    master = _dev(theta)
    w = ctx.gate_train(_dev(X), _dev(t), master, epochs=1, batch=512, lr=1e-3, seed=1)
    step = master.cpu().numpy() - theta
    big = np.abs(g) > 1e-5
    assert big.sum() > 1000
    assert np.allclose(step[big], -1e-3 * np.sign(g[big]), rtol=0, atol=2e-5)
    assert (w.cpu().numpy().view(np.uint16) == mlp.to_bf16_bits(master.cpu().numpy())).all()


def _oracle_gated(img, p, theta):
    """Oracle's own gate: features at the gate point, its own network, a
    threshold placed in the widest gap near the median logit."""
    gx, gy = oracle.grid(img.shape[1], img.shape[0], p["K"])
    p0 = dict(p, levels=p["levels"][:1], gate_level=-1)
    lab0, s0, _, _, mov0 = oracle.segment(img, p0, track=True)
    Xo = oracle.features(img, lab0, p["levels"][0][0] * p["levels"][0][1][-1], s0, mov0, gx, gy)
    z, _ = mlp.forward(theta.astype(np.float64), Xo.astype(np.float64), bf16=True)
    zs = np.sort(z)
    mid = len(zs) // 2
    lo, hi = max(1, mid - len(zs) // 4), min(len(zs) - 1, mid + len(zs) // 4)
    gaps = zs[lo:hi + 1] - zs[lo - 1:hi]
    j = int(np.argmax(gaps)) + lo
    thresh = float((zs[j - 1] + zs[j]) / 2)
    assert gaps.max() > 2e-2, "no clear threshold"
    bits = (z >= thresh).astype(np.uint8)
    lab, _, rep = oracle.segment(img, p, gate=bits)
    return thresh, bits, lab, rep, Xo


def test_gated_segment_matches_oracle(ctx):
    img, p = _he_case()
    theta, wb = _rand_model(21)
    thresh, bits, ref, ref_rep, Xo = _oracle_gated(img, p, theta)
    _say("case: gated 256x192, thresh %.4f, marked %d of %d" % (thresh, bits.sum(), len(bits)))
    labs, reps, X, g = ctx.segment_gated([_dev(img)], p, _dev(wb), thresh, features=True)
    assert np.abs(X.cpu().numpy() - Xo).max() <= 1e-6
    assert (g.cpu().numpy() == bits).all()
    assert (labs[0].cpu().numpy() == ref).all()
    assert reps[0] == ref_rep


def test_gate_with_targets_is_plain_gpu(ctx):
    import torch
    img, p = _he_case()
    gx, gy = oracle.grid(256, 192, 48)
    K = gx * gy
    st = ctx.state(_dev(img), p)
    involved = torch.zeros(K, dtype=torch.uint8, device="cuda")
    st.refine_level(0)
    st.track(involved, None)
    st.refine_level(1)
    st.refine_level(2)
    plain, _ = st.export()
    st.close()
    lab, _ = ctx.segment(_dev(img), p, gate=involved)
    assert (lab.cpu().numpy() == plain.cpu().numpy()).all()


def test_non_finite_model_falls_back_to_plain(ctx, gpu_lib):
    import torch
    img, p = _he_case()
    theta, wb = _rand_model(2)
    wb = wb.copy()
    wb[100] = np.int16(0x7FC0)   # NaN
    lab = torch.empty((192, 256), dtype=torch.int32, device="cuda")
    with pytest.raises(gpu_lib.RapidError) as e:
        ctx.segment_gated([_dev(img)], p, _dev(wb), 0.0, labels=[lab])
    assert e.value.code == -5
    plain, _ = ctx.segment(_dev(img), p)
    assert (lab.cpu().numpy() == plain.cpu().numpy()).all()


@pytest.mark.parametrize("r", [0, 2, 4])
def test_boundary_miss_matches_oracle(ctx, r):
    """Per-label misses and totals of the boundary-recall kernel equal the
    pixel-by-pixel reference, on maps of ragged size (not multiples of the
    64 x 16 tiles), in strided views, with some labels outside [0, K)."""
    import torch
    rng = np.random.default_rng(40 + r)
    H, W, K = 77, 301, 60
    a = np.kron(rng.integers(0, K, size=(20, 60)), np.ones((5, 6), np.int64))[:H, :W].astype(np.int32)
    b = np.kron(rng.integers(0, K, size=(16, 40)), np.ones((6, 8), np.int64))[:H, :W].astype(np.int32)
    b[3:9, 100:140] = K + 5      # out of range: never charged
    b[50:60, 7:30] = -1
    _say("case: boundary miss %dx%d r=%d" % (W, H, r))
    big_a = torch.zeros((H, W + 13), dtype=torch.int32, device="cuda")
    big_b = torch.zeros((H, W + 13), dtype=torch.int32, device="cuda")
    big_a[:, :W] = torch.from_numpy(a).cuda()
    big_b[:, :W] = torch.from_numpy(b).cuda()
    miss, nb, nm = ctx.boundary_miss(big_a[:, :W], big_b[:, :W], radius=r, K=K)
    mo, nbo, nmo = targets.boundary_miss(a, b, r, K)
    assert (nb, nm) == (nbo, nmo)
    assert nm > 0
    assert (miss.cpu().numpy() == mo).all()


def test_learned_gate_beats_random_gate(ctx):
    """What the trained network gains over the method without it.  Trained
    on four 1024^2 H&E tiles (targets: superpixels whose boundary still
    moves by more than 2 px in the gated level), then on a held-out tile the
    network's choice of the 30% of superpixels to refine recovers more of
    the plain result's boundaries than the same number chosen at random, and
    more than refining none."""
    import torch
    from paper_1704_02083_amd import gate, params, synth_gpu
    p = params.gated(1024, 1024, 1024, rule="both")
    tiles = [synth_gpu.he_slide(1024, 1024, seed=300 + i, background=0.4, device="cuda") for i in range(4)]
    X, t = gate.training_set(ctx, tiles, p)
    _say("case: learned gate, %d samples, positive %.3f" % (X.shape[0], t.float().mean().item()))
    _, w = gate.train(ctx, X, t, epochs=20, batch=1024, seed=0)
    rgb = synth_gpu.he_slide(1024, 1024, seed=399, background=0.4, device="cuda")
    plain, _ = ctx.segment(rgb, p, report=False)
    _, _, Xe, _ = ctx.segment_gated([rgb], p, w, 0.0, features=True, report=False)
    z, _ = ctx.mlp_forward(Xe, w, 0.0)
    th = float(torch.quantile(z, 0.7).item())
    labs, _, _, g = ctx.segment_gated([rgb], p, w, th, report=False)
    m = int(g.sum().item())
    K = g.numel()
    assert 0.2 * K < m < 0.4 * K
    br_learned = gate.boundary_recall(ctx, plain, labs[0])
    rng = np.random.default_rng(7)
    brs_random = []
    for _ in range(3):
        rb = np.zeros(K, np.uint8)
        rb[rng.choice(K, m, replace=False)] = 1
        lab_r, _ = ctx.segment(rgb, p, gate=_dev(rb), report=False)
        brs_random.append(gate.boundary_recall(ctx, plain, lab_r))
    lab_0, _ = ctx.segment(rgb, p, gate=torch.zeros(K, dtype=torch.uint8, device="cuda"), report=False)
    br_none = gate.boundary_recall(ctx, plain, lab_0)
    _say("BR learned %.5f random %s none %.5f (marked %d of %d)" % (br_learned, brs_random, br_none, m, K))
    assert br_learned > max(brs_random)
    assert br_learned > br_none


def test_roi_gate_matches_oracle_and_finds_tissue(ctx):
    """The paper's prediction step: a classifier (the gate network trained
    on "most pixels are tissue") labels superpixels at the second level and
    only pairs across the predicted border refine (rule differ).  The gated
    labels equal the oracle run with the same gate bits, and the ROI mask
    (each pixel takes its superpixel's class) recovers the generator's
    tissue mask."""
    import torch
    from paper_1704_02083_amd import gate, synth_gpu
    p = params.default_params(512, 512, 256, levels=params.THREE_LEVEL, gate_level=1)
    p["gate_rule"] = "differ"
    Xs, ts = [], []
    for i in range(4):
        rgb = synth_gpu.he_slide(512, 512, seed=600 + i, background=0.4, device="cuda")
        X, t = gate.roi_samples(ctx, rgb, synth_gpu.tissue_mask(512, 512, seed=600 + i, background=0.4), p)
        Xs.append(X)
        ts.append(t)
    _, w = gate.train(ctx, torch.cat(Xs), torch.cat(ts), epochs=20, batch=512, seed=0)
    rgb = synth_gpu.he_slide(512, 512, seed=699, background=0.4, device="cuda")
    labs, _, _, g = ctx.segment_gated([rgb], p, w, 0.0, report=False)
    _say("case: roi gate 512^2, ROI superpixels %d of %d" % (int(g.sum().item()), g.numel()))
    ref, _, _ = oracle.segment(rgb.cpu().numpy(), p, gate=g.cpu().numpy())
    assert (labs[0].cpu().numpy() == ref).all()
    sc = gate.roi_scores(gate.roi_mask(labs[0], g), synth_gpu.tissue_mask(512, 512, seed=699, background=0.4))
    _say("ROI %s" % sc)
    assert sc["f1"] >= 0.9


def test_gated_batch_of_128_matches_oracle(ctx):
    """128 images in one gated launch: the refinement kernel builds the
    block-sum pyramids (and the gate's second moments) itself from this many
    jobs.  Every image's labels equal the oracle run with the GPU's gate
    bits, and the features of a sample of images equal the oracle's."""
    import torch
    imgs = [synth.he_tile(160, 128, seed=700 + i) for i in range(128)]
    p = params.default_params(160, 128, 20, levels=params.THREE_LEVEL, gate_level=1)
    gx, gy = oracle.grid(160, 128, 20)
    K = gx * gy
    theta, wb = _rand_model(31)
    _say("case: gated batch of 128 images 160x128")
    labs, _, X, g = ctx.segment_gated([_dev(im) for im in imgs], p, _dev(wb), 0.0, features=True,
                                      report=False)
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    X = X.cpu().numpy()
    assert 0 < g.sum() < len(g)
    bad = []
    for i, im in enumerate(imgs):
        ref, _, _ = oracle.segment(im, p, gate=g[i * K:(i + 1) * K])
        if not (labs[i].cpu().numpy() == ref).all():
            bad.append(i)
    assert not bad, "images differ: %s" % bad[:10]
    p0 = dict(p, levels=p["levels"][:1], gate_level=-1)
    for i in (0, 63, 127):
        lab0, s0, _, _, mov0 = oracle.segment(imgs[i], p0, track=True)
        Xo = oracle.features(imgs[i], lab0, 16, s0, mov0, gx, gy)
        assert np.abs(X[i * K:(i + 1) * K] - Xo).max() <= 1e-6


def test_state_gate_matches_oracle_and_fused(ctx):
    """rapid_gate on a level-by-level state (moved pixels tracked from the
    first level) decides the same bits as the oracle's features and network
    and as the single-launch gated path; the levels refined under those bits
    match both."""
    import torch
    img, p = _he_case()
    theta, wb = _rand_model(21)
    thresh, bits, ref, ref_rep, Xo = _oracle_gated(img, p, theta)
    K = len(bits)
    _say("case: rapid_gate level by level 256x192, marked %d of %d" % (bits.sum(), K))
    st = ctx.state(_dev(img), p)
    moved = torch.zeros(K, dtype=torch.int64, device="cuda")
    st.track(None, moved)
    reps = st.refine_level(0)
    g, X = st.gate(_dev(wb), thresh, features=True)
    assert np.abs(X.cpu().numpy() - Xo).max() <= 1e-6
    assert (g.cpu().numpy() == bits).all()
    st.track(None, None)
    reps += st.refine_level(1, gate=g)
    reps += st.refine_level(2, gate=g)
    lab, _ = st.export()
    assert (lab.cpu().numpy() == ref).all()
    assert reps == ref_rep
    st.close()
    labs, _, Xf, gf = ctx.segment_gated([_dev(img)], p, _dev(wb), thresh, features=True)
    assert (gf.cpu().numpy() == bits).all()
    assert (Xf.cpu().numpy() == X.cpu().numpy()).all()
    assert (labs[0].cpu().numpy() == ref).all()


def test_state_gate_refuses_non_finite_model(ctx, gpu_lib):
    import torch
    img, p = _he_case()
    _, wb = _rand_model(2)
    wb = wb.copy()
    wb[7] = np.int16(0x7F80)   # +inf
    st = ctx.state(_dev(img), p)
    st.refine_level(0)
    g = torch.zeros(st.K, dtype=torch.uint8, device="cuda")
    with pytest.raises(gpu_lib.RapidError) as e:
        st.gate(_dev(wb), 0.0, out=g)
    assert e.value.code == -5
    assert (g.cpu().numpy() == 1).all()
    st.close()


@pytest.mark.parametrize("res", [0, 1, 2, 3])
def test_gated_segment_every_residency(gpu_lib, res):
    """The single-launch gated path with the per-superpixel state all in
    global memory (0), all in LDS (1), only the means records in LDS (2) or
    the means records and flow counters (3):
    the gate point borrows the LDS that holds no statistics, so every
    residency must still give the oracle's features, bits and labels."""
    import os
    img, p = _he_case()
    theta, wb = _rand_model(21)
    thresh, bits, ref, ref_rep, Xo = _oracle_gated(img, p, theta)
    old = os.environ.get("RAPID_SHAPE")
    os.environ["RAPID_SHAPE"] = "1024,%d,1" % res
    try:
        c = gpu_lib.Context(0, timing=True)
        _say("case: gated 256x192, residency %d" % res)
        labs, reps, X, g = c.segment_gated([_dev(img)], p, _dev(wb), thresh, features=True)
        assert c.last_timings()["stats_lds"] == res
        assert np.abs(X.cpu().numpy() - Xo).max() <= 1e-6
        assert (g.cpu().numpy() == bits).all()
        assert (labs[0].cpu().numpy() == ref).all()
        assert reps[0] == ref_rep
        c.close()
    finally:
        if old is None:
            os.environ.pop("RAPID_SHAPE", None)
        else:
            os.environ["RAPID_SHAPE"] = old


def test_gated_large_grid_matches_oracle(ctx):
    """1024 x 768 H&E tile with K = 3072: the state does not fit LDS whole,
    so the launch keeps only the means records there (the gate point then
    works in the rest).  Features against the oracle's; bits against the
    oracle's network wherever its logit is clear of the threshold (bf16
    rounding moves logits by up to 1e-2); labels against the oracle run
    under the GPU's own bits."""
    img = synth.he_tile(1024, 768, seed=31)
    p = params.default_params(1024, 768, 3072, levels=params.THREE_LEVEL, gate_level=1)
    theta, wb = _rand_model(22)
    gx, gy = oracle.grid(1024, 768, 3072)
    p0 = dict(p, levels=p["levels"][:1], gate_level=-1)
    lab0, s0, _, _, mov0 = oracle.segment(img, p0, track=True)
    Xo = oracle.features(img, lab0, 16, s0, mov0, gx, gy)
    z, _ = mlp.forward(theta.astype(np.float64), Xo.astype(np.float64), bf16=True)
    thresh = float(np.median(z))
    _say("case: gated 1024x768 K=%d" % len(z))
    labs, reps, X, g = ctx.segment_gated([_dev(img)], p, _dev(wb), thresh, features=True)
    assert np.abs(X.cpu().numpy() - Xo).max() <= 1e-6
    g = g.cpu().numpy()
    far = np.abs(z - thresh) > 1e-2
    assert far.sum() > 0.9 * len(z)
    assert (g[far] == (z[far] >= thresh)).all()
    ref, _, ref_rep = oracle.segment(img, p, gate=g)
    assert (labs[0].cpu().numpy() == ref).all()
    assert reps[0] == ref_rep


@pytest.mark.parametrize("rule", ["either", "both", "differ"])
def test_gated_nothing_marked_matches_oracle(ctx, rule):
    """No superpixel marked (threshold above every logit): no pair is active
    in the gated stages, the last one runs no sweep and the output comes
    from the previous stage's map; labels and stage counters must still be
    the oracle's under an all-zero gate."""
    img, p = _he_case()
    p = dict(p, gate_rule=rule)
    _, wb = _rand_model(21)
    K = oracle.n_superpixels(256, 192, p)
    ref, _, ref_rep = oracle.segment(img, p, gate=np.zeros(K, np.uint8))
    _say("case: gated, nothing marked, rule %s" % rule)
    labs, reps, _, g = ctx.segment_gated([_dev(img)], p, _dev(wb), 1e9)
    assert int(g.sum().item()) == 0
    assert (labs[0].cpu().numpy() == ref).all()
    assert reps[0] == ref_rep
    # and through the caller-supplied gate of rapid_segment
    lab, rep = ctx.segment(_dev(img), p, gate=_dev(np.zeros(K, np.uint8)))
    assert (lab.cpu().numpy() == ref).all() and rep == ref_rep
