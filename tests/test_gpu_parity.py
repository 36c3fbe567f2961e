"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

Labels and statistics are integers, so the bar is bit-exact equality of the
label map, the per-superpixel statistics and every per-stage counter.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1704_02083_amd import params, synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0)
    yield c
    c.close()


def _gpu_segment(ctx, img, p, gate=None):
    import torch
    rgb = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    g = None if gate is None else torch.from_numpy(gate.astype(np.uint8)).cuda()
    lab, rep = ctx.segment(rgb, p, gate=g)
    torch.cuda.synchronize()
    return lab.cpu().numpy(), rep


def _assert_same(got, rep, ref, ref_rep, what):
    mism = int((got != ref).sum())
    assert mism == 0, "%s: %d labels differ" % (what, mism)
    assert rep == ref_rep, "%s: stage counters differ\n%s\n%s" % (what, rep, ref_rep)


def test_config1_bit_exact(ctx):
    _say("case: config1 256x256 K=64")
    img = synth.voronoi_blur()
    p = params.config1()
    got, rep = _gpu_segment(ctx, img, p)
    ref, _, ref_rep = oracle.segment(img, p)
    _assert_same(got, rep, ref, ref_rep, "config1")


CASES = [
    # W, H, K, levels, min, seed
    (64, 64, 4, [(1, [16, 8, 4, 2, 1])], 0, 1),
    (97, 61, 12, [(1, [8, 4, 2, 1])], 10, 2),          # ragged edges on both axes
    (33, 17, 2, [(1, [16, 8, 4, 2, 1])], 0, 3),         # 1-px edge column and row
    (200, 40, 20, [(1, [8, 4, 2, 1])], 5, 4),
    (128, 96, 24, params.THREE_LEVEL, 64, 5),          # three levels, ratio 4
    (17, 300, 6, [(1, [4, 2, 1])], 3, 6),
    (64, 64, 1, [(1, [16, 8, 4, 2, 1])], 0, 7),         # one superpixel: no boundary
    (16, 16, 1, [(1, [1])], 0, 8),                      # single stage at B = 1
    (1, 64, 4, [(1, [1])], 0, 21),                      # one pixel wide
    (64, 1, 4, [(1, [1])], 0, 22),                      # one pixel tall
    (2, 300, 8, [(1, [2, 1])], 0, 23),                  # two pixels wide, blocks clipped to the image
    (300, 2, 8, [(1, [2, 1])], 0, 24),
]


@pytest.mark.parametrize("W,H,K,levels,mn,seed", CASES)
def test_small_cases_bit_exact(ctx, W, H, K, levels, mn, seed):
    _say("case: %dx%d K=%d seed=%d" % (W, H, K, seed))
    img = synth.voronoi_blur(W, H, regions=max(3, K // 2), seed=seed)
    p = params.default_params(W, H, K, levels=levels, min_size=mn)
    got, rep = _gpu_segment(ctx, img, p)
    ref, _, ref_rep = oracle.segment(img, p)
    _assert_same(got, rep, ref, ref_rep, "small %dx%d" % (W, H))


@pytest.mark.parametrize("seed", [11, 12, 13, 14])
def test_random_weights_bit_exact(ctx, seed):
    rng = np.random.default_rng(seed)
    W, H = int(rng.integers(24, 140)), int(rng.integers(24, 140))
    K = int(rng.integers(2, 30))
    _say("case: random weights %dx%d K=%d seed=%d" % (W, H, K, seed))
    img = synth.voronoi_gradient(W, H, seed=seed, regions=(3, 12))
    p = params.default_params(W, H, K, levels=[(1, [4, 2, 1])])
    p.update(w_col=int(rng.integers(0, 4000)), w_pos=int(rng.integers(0, 3000)),
             w_bnd=int(rng.integers(0, 1 << 20)), frac_bits=int(rng.integers(0, 5)),
             min_size=int(rng.integers(0, 60)), max_size=int(rng.integers(60, 4000)),
             max_sweeps=int(rng.integers(1, 40)))
    try:
        oracle_out = oracle.segment(img, p)
    except RuntimeError:
        pytest.skip("grid does not fit")
    got, rep = _gpu_segment(ctx, img, p)
    _assert_same(got, rep, oracle_out[0], oracle_out[2], "random weights")


@pytest.mark.parametrize("rule", ["either", "both", "differ"])
def test_gate_bit_exact(ctx, rule):
    """A seeded gate (input to both sides) restricts moves past the gate
    level (Eq. (7)) under each pair rule; labels and counters must still
    agree exactly."""
    img = synth.voronoi_blur(160, 128, regions=14, seed=21)
    p = params.default_params(160, 128, 20, levels=params.THREE_LEVEL, gate_level=1)
    p["gate_rule"] = rule
    K = oracle.n_superpixels(160, 128, p)
    gate = (np.random.default_rng(4).random(K) < (0.4 if rule == "either" else 0.7)).astype(np.uint8)
    _say("case: gate %s 160x128 K=%d marked=%d" % (rule, K, int(gate.sum())))
    got, rep = _gpu_segment(ctx, img, p, gate=gate)
    ref, _, ref_rep = oracle.segment(img, p, gate=gate)
    _assert_same(got, rep, ref, ref_rep, "gate")


def test_gate_beyond_lds_bitmap_refused(ctx, gpu_lib):
    """A gated run keeps one bit per superpixel in LDS (at most 2^18
    superpixels per image); a larger grid is refused before any launch."""
    import torch
    W = H = 1040
    p = {"K": 0, "gx": 520, "gy": 520, "levels": [(1, [2, 1])], "gate_level": 0, "frac_bits": 4,
         "max_sweeps": 4, "min_size": 0, "max_size": 64, "w_col": 1, "w_pos": 1, "w_bnd": 1}
    rgb = torch.zeros((H, W, 3), dtype=torch.uint8, device="cuda")
    gate = torch.ones(520 * 520, dtype=torch.uint8, device="cuda")
    with pytest.raises(gpu_lib.RapidError) as e:
        ctx.segment(rgb, p, gate=gate)
    assert e.value.code == -1


def test_sweep_cap_not_converged(ctx):
    """max_sweeps = 1: the stages stop after one sweep, unconverged, exactly
    as the oracle's."""
    img = synth.voronoi_blur(128, 96, regions=10, seed=5)
    p = params.default_params(128, 96, 24, max_sweeps=1)
    got, rep = _gpu_segment(ctx, img, p)
    ref, _, ref_rep = oracle.segment(img, p)
    _assert_same(got, rep, ref, ref_rep, "max_sweeps 1")
    assert any(r["converged"] == 0 for r in rep)


def test_state_api_level_by_level(ctx):
    """state_create + refine_level per level + export equals the oracle, and
    the exported statistics equal the oracle's (reuse across levels)."""
    import torch
    img = synth.voronoi_blur(192, 160, regions=12, seed=31)
    p = params.default_params(192, 160, 30, levels=params.THREE_LEVEL)
    _say("case: state api 192x160")
    st = ctx.state(torch.from_numpy(img).cuda(), p)
    reps = []
    for l in range(3):
        reps += st.refine_level(l)
    lab, stats = st.export()
    torch.cuda.synchronize()
    ref, ref_stats, ref_rep = oracle.segment(img, p)
    _assert_same(lab.cpu().numpy(), reps, ref, ref_rep, "state api")
    assert (stats.cpu().numpy() == ref_stats).all()
    st.close()


@pytest.mark.parametrize("with_stats", [True, False])
def test_state_checkpoint_resume(ctx, with_stats):
    """Export after level 1 of three, import into a fresh state (statistics
    given, or rebuilt from the image), refine the remaining levels: labels,
    statistics and stage counters equal the uninterrupted oracle run."""
    import torch
    img = synth.voronoi_blur(192, 160, regions=12, seed=33)
    p = params.default_params(192, 160, 30, levels=params.THREE_LEVEL)
    _say("case: checkpoint after level 1, stats given %s" % with_stats)
    rgb = torch.from_numpy(img).cuda()
    a = ctx.state(rgb, p)
    reps = a.refine_level(0)
    lab1, stats1 = a.export()
    a.close()
    b = ctx.state(rgb, p)
    b.import_(1, lab1, stats1 if with_stats else None)
    lab_b, stats_b = b.export()
    torch.cuda.synchronize()
    assert (lab_b.cpu().numpy() == lab1.cpu().numpy()).all()
    assert (stats_b.cpu().numpy() == stats1.cpu().numpy()).all()
    reps += b.refine_level(1)
    reps += b.refine_level(2)
    lab, stats = b.export()
    torch.cuda.synchronize()
    ref, ref_stats, ref_rep = oracle.segment(img, p)
    _assert_same(lab.cpu().numpy(), reps, ref, ref_rep, "checkpoint resume")
    assert (stats.cpu().numpy() == ref_stats).all()
    # a finished state restores too: export of the import is the input
    c = ctx.state(rgb, p)
    c.import_(3, lab, None)
    lab_c, stats_c = c.export()
    torch.cuda.synchronize()
    assert (lab_c.cpu().numpy() == ref).all() and (stats_c.cpu().numpy() == ref_stats).all()
    c.close()
    b.close()


def test_state_import_rejects_bad_labels(ctx, gpu_lib):
    """Labels that are not constant on the point's blocks, or out of range,
    are refused; the state is unusable until a valid import."""
    import torch
    img = synth.voronoi_blur(128, 96, regions=8, seed=34)
    p = params.default_params(128, 96, 12, levels=params.THREE_LEVEL)
    rgb = torch.from_numpy(img).cuda()
    st = ctx.state(rgb, p)
    st.refine_level(0)
    lab1, stats1 = st.export()
    bad = lab1.clone()
    bad[17, 21] = (int(bad[17, 21]) + 1) % st.K     # inside a 16 x 16 block
    with pytest.raises(gpu_lib.RapidError) as e:
        st.import_(1, bad)
    assert e.value.code == -1
    with pytest.raises(gpu_lib.RapidError) as e:
        st.refine_level(1)
    assert e.value.code == -4
    neg = lab1.clone()
    neg[:16, :16] = st.K                             # a whole block out of range
    with pytest.raises(gpu_lib.RapidError) as e:
        st.import_(1, neg)
    assert e.value.code == -1
    with pytest.raises(gpu_lib.RapidError) as e:
        st.import_(4, lab1)                          # beyond the last level
    assert e.value.code == -1
    st.import_(1, lab1, stats1)
    st.refine_level(1)
    st.close()


def test_state_api_rejects_out_of_order(ctx, gpu_lib):
    import torch
    img = synth.voronoi_blur(64, 64, regions=5, seed=2)
    p = params.default_params(64, 64, 4, levels=params.THREE_LEVEL)
    st = ctx.state(torch.from_numpy(img).cuda(), p)
    with pytest.raises(gpu_lib.RapidError) as e:
        st.refine_level(1)
    assert e.value.code == -4
    st.close()


def test_invalid_params_rejected_without_launch(ctx, gpu_lib):
    import torch
    img = torch.zeros((64, 64, 3), dtype=torch.uint8, device="cuda")
    p = params.default_params(64, 64, 4)
    p["levels"] = [(1, [8, 16])]
    with pytest.raises(gpu_lib.RapidError) as e:
        ctx.segment(img, p)
    assert e.value.code == -1


def test_batch_bsd_shaped_sample(ctx):
    """The batched workload (100 images 481x321 + 100 of 321x481, K = 400)
    in the launch the benchmark times; a sample of the images is compared
    with independent oracle runs."""
    import torch
    imgs = synth.batch_images(200)
    rgbs = [torch.from_numpy(im).cuda() for im in imgs]
    W, H = 481, 321
    p = params.config2(W, H)
    _say("case: batch of 200, launching")
    labs, reps = ctx.segment_batch(rgbs, p)
    torch.cuda.synchronize()
    for i in (0, 1, 57, 99, 100, 143, 199):
        _say("case: batch image %d" % i)
        ref, _, ref_rep = oracle.segment(imgs[i], p)
        _assert_same(labs[i].cpu().numpy(), reps[i], ref, ref_rep, "batch image %d" % i)


def test_determinism_and_thread_counts(gpu_lib):
    """Repeated runs and other workgroup sizes give identical labels."""
    import torch
    img = synth.voronoi_gradient(321, 481, seed=1150)
    p = params.config2(321, 481)
    rgb = torch.from_numpy(img).cuda()
    outs = []
    old = os.environ.get("RAPID_THREADS")
    try:
        for t in ("256", "512", "1024", "512"):
            os.environ["RAPID_THREADS"] = t
            c = gpu_lib.Context(0)
            _say("case: threads %s" % t)
            lab, rep = c.segment(rgb, p)
            torch.cuda.synchronize()
            outs.append((lab.cpu().numpy(), rep))
            c.close()
    finally:
        if old is None:
            os.environ.pop("RAPID_THREADS", None)
        else:
            os.environ["RAPID_THREADS"] = old
    for lab, rep in outs[1:]:
        assert (lab == outs[0][0]).all() and rep == outs[0][1]


def test_int64_and_fp64_energy_paths(ctx):
    """2000x64 image, blocks 64..1 and w_pos = 100: the worst-case block
    energy exceeds 2^53 at B >= 8 (exact int64 evaluation) and stays below it
    at B <= 4 (exact fp64 evaluation); both must match the oracle."""
    img = synth.voronoi_gradient(2000, 64, seed=77, regions=(20, 40))
    p = params.default_params(2000, 64, 20, levels=[(1, [64, 32, 16, 8, 4, 2, 1])], min_size=100)
    p.update(w_col=50, w_pos=100, w_bnd=4096)
    _say("case: 2000x64 int64 and fp64 energy paths")
    got, rep = _gpu_segment(ctx, img, p)
    ref, _, ref_rep = oracle.segment(img, p)
    _assert_same(got, rep, ref, ref_rep, "int64/fp64 paths")


def test_timing_history_of_back_to_back_calls(gpu_lib):
    """rapid_timing_history returns one refinement-kernel duration per timed
    call queued back to back (oldest first), the last equal to
    rapid_last_timings; at most the ring's 128."""
    import torch
    img = synth.voronoi_blur(256, 256, regions=24, seed=1)
    p = params.config1()
    rgb = torch.from_numpy(img).cuda()
    c = gpu_lib.Context(0, timing=True)
    try:
        lab = torch.empty((256, 256), dtype=torch.int32, device="cuda")
        for _ in range(5):
            c.segment(rgb, p, labels=lab, report=False)
        h = c.timing_history(8)
        assert len(h) == 5 and all(x > 0 for x in h)
        assert h[-1] == c.last_timings()["refine_ms"]
        for _ in range(130):
            c.segment(rgb, p, labels=lab, report=False)
        h = c.timing_history(200)
        assert len(h) == 128 and all(x > 0 for x in h)
        ref, _, _ = oracle.segment(img, p)
        assert (lab.cpu().numpy() == ref).all()
    finally:
        c.close()
