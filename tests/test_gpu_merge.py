"""GPU parity of merge on underflow (Sec. 3.1, Eqs. (4)-(5)) against the
CPU oracle: labels, statistics and every stage counter (merges included)
bit-exact, with the statistics in LDS and in global memory, under a gate,
level by level, and in the single-launch gated path."""
import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_1704_02083_amd import params, synth

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


def _check(ctx, img, p, gate=None, what=""):
    import torch
    g = None if gate is None else _dev(gate.astype(np.uint8))
    lab, rep = ctx.segment(_dev(img), p, gate=g)
    torch.cuda.synchronize()
    ref, ref_stats, ref_rep = oracle.segment(img, p, gate=gate)
    mism = int((lab.cpu().numpy() != ref).sum())
    assert mism == 0, "%s: %d labels differ" % (what, mism)
    assert rep == ref_rep, "%s: stage counters differ\n%s\n%s" % (what, rep, ref_rep)
    return ref_rep


def _merge_params(W, H, K, levels, div):
    p = params.default_params(W, H, K, levels=levels)
    A = (W * H) // oracle.n_superpixels(W, H, p)
    p.update(min_size=A // div, merge=True)
    return p


def test_merge_three_cells_gpu(ctx):
    """The hand-traced case of the oracle's pins: cells 0 and 1 merge, 2
    stays (its merged size would pass max_size)."""
    rgb = np.zeros((4, 12, 3), np.uint8)
    rgb[:, 0:4] = (200, 0, 0)
    rgb[:, 4:8] = (190, 10, 0)
    rgb[:, 8:12] = (0, 0, 200)
    p = {"K": 0, "gx": 3, "gy": 1, "levels": [(1, [4])], "gate_level": -1, "frac_bits": 0,
         "max_sweeps": 16, "min_size": 8, "max_size": 40, "w_col": 1, "w_pos": 0, "w_bnd": 0,
         "merge": True}
    _say("case: merge three cells")
    rep = _check(ctx, rgb, p, what="three cells")
    assert rep[0]["merges"] == 1


CASES = [
    # W, H, K, levels, min_size divisor, seed
    (128, 96, 24, [(1, [8, 4, 2, 1])], 4, 1),
    (160, 128, 40, params.THREE_LEVEL, 4, 2),
    (97, 61, 12, [(1, [8, 4, 2, 1])], 3, 3),          # ragged edges
    (120, 80, 30, [(1, [4, 2, 1])], 2, 4),
    (200, 40, 20, [(1, [8, 4, 2, 1])], 2, 5),
]


@pytest.mark.parametrize("W,H,K,levels,div,seed", CASES)
def test_merge_bit_exact(ctx, W, H, K, levels, div, seed):
    img = synth.voronoi_blur(W, H, regions=max(3, K // 2), seed=seed)
    p = _merge_params(W, H, K, levels, div)
    _say("case: merge %dx%d K=%d min=%d seed=%d" % (W, H, K, p["min_size"], seed))
    rep = _check(ctx, img, p, what="merge %dx%d" % (W, H))
    assert sum(r["merges"] for r in rep) > 0


def test_merge_global_statistics(ctx):
    """512 x 512, K = 4096: the statistics do not fit LDS and live in global
    memory; merges must still agree exactly."""
    img = synth.voronoi_gradient(512, 512, seed=41, regions=(200, 400))
    p = _merge_params(512, 512, 4096, [(1, [8, 4, 2, 1])], 3)
    _say("case: merge 512x512 K=4096 global statistics")
    rep = _check(ctx, img, p, what="merge global")
    assert sum(r["merges"] for r in rep) > 0


def test_merge_batch_bsd_shaped(ctx):
    """Batched launch (LDS statistics, the block-sum pyramid built in the
    launch for 128+ images) with merges; a sample compared with the oracle."""
    import torch
    imgs = synth.batch_images(128)
    p = dict(params.config2(481, 321), merge=True)
    _say("case: merge batch of 128")
    labs, reps = ctx.segment_batch([_dev(im) for im in imgs], p)
    torch.cuda.synchronize()
    for i in (0, 63, 100, 127):
        ref, _, ref_rep = oracle.segment(imgs[i], p)
        assert (labs[i].cpu().numpy() == ref).all(), i
        assert reps[i] == ref_rep, i
        assert sum(r["merges"] for r in ref_rep) > 0


@pytest.mark.parametrize("rule,seed", [("either", 23), ("both", 24)])
def test_merge_under_gate(ctx, rule, seed):
    """Past the gate level only pairs the gate activates may merge."""
    img = synth.voronoi_blur(160, 128, regions=14, seed=seed)
    p = _merge_params(160, 128, 40, params.THREE_LEVEL, 2)
    p.update(gate_level=1, gate_rule=rule)
    K = oracle.n_superpixels(160, 128, p)
    gate = (np.random.default_rng(5).random(K) < 0.6).astype(np.uint8)
    _say("case: merge under gate %s seed %d" % (rule, seed))
    rep = _check(ctx, img, p, gate=gate, what="merge gate %s" % rule)
    assert sum(r["merges"] for r in rep[1:]) > 0


def test_merge_level_by_level(ctx):
    import torch
    img = synth.voronoi_blur(192, 160, regions=12, seed=35)
    p = _merge_params(192, 160, 30, params.THREE_LEVEL, 3)
    _say("case: merge level by level")
    st = ctx.state(_dev(img), p)
    reps = []
    for l in range(3):
        reps += st.refine_level(l)
    lab, stats = st.export()
    torch.cuda.synchronize()
    ref, ref_stats, ref_rep = oracle.segment(img, p)
    assert (lab.cpu().numpy() == ref).all()
    assert (stats.cpu().numpy() == ref_stats).all()
    assert reps == ref_rep
    st.close()


def test_merge_fused_gate(ctx):
    """Single-launch gated path with merges before and after the gate: the
    oracle's features (zeros for merged superpixels) and network give the
    same bits and labels."""
    img = synth.he_tile(256, 192, seed=12)
    p = _merge_params(256, 192, 48, params.THREE_LEVEL, 4)
    p["gate_level"] = 1
    theta = mlp.he_init(21).astype(np.float32)
    wb = mlp.to_bf16_bits(theta).view(np.int16)
    gx, gy = oracle.grid(256, 192, 48)
    p0 = dict(p, levels=p["levels"][:1], gate_level=-1)
    lab0, s0, rep0, _, mov0 = oracle.segment(img, p0, track=True)
    Xo = oracle.features(img, lab0, 16, s0, mov0, gx, gy)
    z, _ = mlp.forward(theta.astype(np.float64), Xo.astype(np.float64), bf16=True)
    zs = np.sort(z)
    gaps = zs[1:] - zs[:-1]
    mid = len(zs) // 2
    j = int(np.argmax(gaps[mid // 2: mid + mid // 2])) + mid // 2
    thresh = float((zs[j] + zs[j + 1]) / 2)
    assert gaps[j] > 1e-2, "no clear threshold"
    bits = (z >= thresh).astype(np.uint8)
    ref, _, ref_rep = oracle.segment(img, p, gate=bits)
    _say("case: merge fused gate, merges before the gate %d" % sum(r["merges"] for r in rep0))
    labs, reps, X, g = ctx.segment_gated([_dev(img)], p, _dev(wb), thresh, features=True)
    assert np.abs(X.cpu().numpy() - Xo).max() <= 1e-6
    assert (g.cpu().numpy() == bits).all()
    assert (labs[0].cpu().numpy() == ref).all()
    assert reps[0] == ref_rep
