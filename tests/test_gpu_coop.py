"""One image on many workgroups: the cooperative launch shape, in which the
class phases of a single image are split over G workgroups separated by grid
barriers (and sweeps with at most S active blocks run on one workgroup),
gives the labels, statistics and stage counters of the oracle bit for bit,
at every G and S, and falls back to one workgroup per image where it does not
apply (batches, merge on underflow, gates)."""
import contextlib
import os

import numpy as np
import pytest

import oracle
from paper_1704_02083_amd import params, synth, synth_gpu

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@contextlib.contextmanager
def _shape(groups, solo=-1):
    """Contexts created inside use one image on `groups` workgroups of 1024
    lanes (state in global memory, the block-sum pyramid built over the grid
    inside the launch), sweeps with at most `solo` active blocks on one
    workgroup."""
    old = os.environ.get("RAPID_SHAPE")
    os.environ["RAPID_SHAPE"] = "1024,0,0,%d,%d" % (groups, solo)
    try:
        yield
    finally:
        if old is None:
            os.environ.pop("RAPID_SHAPE", None)
        else:
            os.environ["RAPID_SHAPE"] = old


def _run(ctx, img, p):
    import torch
    rgb = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    lab, rep = ctx.segment(rgb, p)
    torch.cuda.synchronize()
    return lab.cpu().numpy(), rep


CASES = [
    # W, H, K, levels, min, seed
    (64, 64, 4, [(1, [16, 8, 4, 2, 1])], 0, 1),
    (97, 61, 12, [(1, [8, 4, 2, 1])], 10, 2),          # ragged edges on both axes
    (33, 17, 2, [(1, [16, 8, 4, 2, 1])], 0, 3),         # 1-px edge column and row
    (128, 96, 24, params.THREE_LEVEL, 64, 5),          # three levels, ratio 4
    (64, 64, 1, [(1, [16, 8, 4, 2, 1])], 0, 7),         # one superpixel: no boundary
    (16, 16, 1, [(1, [1])], 0, 8),                      # single stage at B = 1
    (481, 321, 400, [(1, [16, 8, 4, 2, 1])], 0, 9),    # a batch image's shape
    (1, 64, 4, [(1, [1])], 0, 21),                      # one pixel wide
    (64, 1, 4, [(1, [1])], 0, 22),                      # one pixel tall
    (2, 300, 8, [(1, [2, 1])], 0, 23),                  # two pixels wide, blocks clipped to the image
    (300, 2, 8, [(1, [2, 1])], 0, 24),
]


def test_coop_small_cases_bit_exact(gpu_lib):
    refs = []
    imgs = []
    for (W, H, K, levels, mn, seed) in CASES:
        img = synth.voronoi_blur(W, H, regions=max(3, K // 2), seed=seed)
        p = params.default_params(W, H, K, levels=levels, min_size=mn)
        ref, _, ref_rep = oracle.segment(img, p)
        imgs.append((img, p))
        refs.append((ref, ref_rep))
    # S = 2^30: every sweep on one workgroup; 4096: the small ones
    for g, so in ((2, -1), (8, -1), (64, -1), (256, -1), (64, 4096), (8, 1 << 30)):
        with _shape(g, so):
            c = gpu_lib.Context(0, timing=True)
        try:
            for (W, H, K, _, _, seed), (img, p), (ref, ref_rep) in zip(CASES, imgs, refs):
                _say("case: coop G=%d S=%d %dx%d K=%d seed=%d" % (g, so, W, H, K, seed))
                got, rep = _run(c, img, p)
                tm = c.last_timings()
                assert tm["workgroups"] == g
                assert tm["pyramid"] == 1   # the whole image in one launch
                mism = int((got != ref).sum())
                assert mism == 0, "G=%d %dx%d: %d labels differ" % (g, W, H, mism)
                assert rep == ref_rep, "G=%d %dx%d: stage counters differ" % (g, W, H)
        finally:
            c.close()


def test_coop_config1_and_he_bit_exact(gpu_lib):
    """The 256^2 image with K = 64, and a 1024 x 768 H&E tile with three
    levels and K = 768, on 8, 64 and 256 workgroups."""
    cases = [(synth.voronoi_blur(), params.config1())]
    he = synth.he_tile(1024, 768, seed=31)
    cases.append((he, params.default_params(1024, 768, 768, levels=params.THREE_LEVEL)))
    refs = [oracle.segment(img, p) for img, p in cases]
    for g in (8, 64, 256):
        with _shape(g):
            c = gpu_lib.Context(0)
        try:
            for i, ((img, p), (ref, _, ref_rep)) in enumerate(zip(cases, refs)):
                _say("case: coop G=%d image %d" % (g, i))
                got, rep = _run(c, img, p)
                assert (got == ref).all() and rep == ref_rep, (g, i)
        finally:
            c.close()


def test_coop_he4096_three_levels_bit_exact(gpu_lib):
    """The 4096^2 H&E tile with K = 16384 and three levels on 64 and 256
    workgroups, and on 32 with sweeps of at most 16384 active blocks on one
    workgroup, equals the oracle."""
    import torch
    rgb = synth_gpu.he_slide(4096, 4096, seed=3, background=0.3, device="cuda")
    p = params.config3()
    ref, _, ref_rep = oracle.segment(rgb.cpu().numpy(), p)
    for g, so in ((64, -1), (256, -1), (32, 16384)):
        with _shape(g, so):
            c = gpu_lib.Context(0, timing=True)
        try:
            _say("case: coop G=%d S=%d 4096^2 K=16384" % (g, so))
            lab, rep = c.segment(rgb, p)
            torch.cuda.synchronize()
            assert c.last_timings()["workgroups"] == g
            mism = int((lab.cpu().numpy() != ref).sum())
            assert mism == 0, "G=%d: %d labels differ" % (g, mism)
            assert rep == ref_rep
        finally:
            c.close()


def test_coop_level_by_level_state(gpu_lib):
    """rapid_state_create and rapid_refine_level per level on 64 workgroups:
    labels, statistics and counters equal the one-workgroup state path, and
    the involvement and moved-pixel tracking match too."""
    import torch
    img = synth.he_tile(512, 384, seed=41)
    p = params.default_params(512, 384, 192, levels=params.THREE_LEVEL)
    rgb = torch.from_numpy(img).cuda()
    out = []
    for g in (1, 64):
        with _shape(g, 8192):
            c = gpu_lib.Context(0)
        try:
            _say("case: level by level, G=%d" % g)
            st = c.state(rgb, p)
            K = st.K
            inv = torch.zeros(K, dtype=torch.uint8, device="cuda")
            mv = torch.zeros(K, dtype=torch.int64, device="cuda")
            st.track(involved=inv, moved=mv)
            reps = st.refine_level(0) + st.refine_level(1) + st.refine_level(2)
            lab, stats = st.export()
            torch.cuda.synchronize()
            out.append((lab.cpu().numpy(), stats.cpu().numpy(), reps, inv.cpu().numpy(), mv.cpu().numpy()))
            st.close()
        finally:
            c.close()
    (l1, s1, r1, i1, m1), (l2, s2, r2, i2, m2) = out
    assert (l1 == l2).all() and (s1 == s2).all() and r1 == r2
    assert (i1 == i2).all() and (m1 == m2).all()
    ref, ref_stats, ref_rep = oracle.segment(img, p)
    assert (l2 == ref).all() and r2 == ref_rep


def test_coop_shape_falls_back_where_it_does_not_apply(gpu_lib):
    """Merge on underflow and batches run one workgroup per image even when
    the cooperative shape is asked for, with the oracle's labels."""
    import torch
    img = synth.voronoi_blur(160, 120, regions=20, seed=51)
    p = params.default_params(160, 120, 40, min_size=120)
    p["merge"] = 1
    ref, _, ref_rep = oracle.segment(img, p)
    with _shape(64):
        c = gpu_lib.Context(0, timing=True)
    try:
        _say("case: coop asked, merge on")
        got, rep = _run(c, img, p)
        assert c.last_timings()["workgroups"] == 1
        assert (got == ref).all() and rep == ref_rep
        _say("case: coop asked, batch of 3")
        imgs = [synth.voronoi_blur(96, 80, regions=10, seed=60 + i) for i in range(3)]
        pb = params.default_params(96, 80, 12)
        labs, reps = c.segment_batch([torch.from_numpy(im).cuda() for im in imgs], pb)
        torch.cuda.synchronize()
        assert c.last_timings()["workgroups"] == 1
        for im, lab, rp in zip(imgs, labs, reps):
            r, _, rr = oracle.segment(im, pb)
            assert (lab.cpu().numpy() == r).all() and rp == rr
    finally:
        c.close()


def test_coop_autotune_single_image(gpu_lib, tmp_path):
    """The autotuner times the cooperative shapes beside the one-workgroup
    shapes for a single plain image; whatever it picks gives the oracle's
    labels, and the choice (with its workgroup count) survives the cache."""
    import torch
    img = synth.he_tile(1024, 1024, seed=61)
    p = params.default_params(1024, 1024, 1024, levels=params.THREE_LEVEL)
    ref, _, ref_rep = oracle.segment(img, p)
    rgb = torch.from_numpy(img).cuda()
    cache = str(tmp_path / "tune.json")
    _say("case: autotune single 1024^2 image")
    c = gpu_lib.Context(0, timing=True, autotune=True, autotune_cache=cache)
    try:
        lab, rep = c.segment(rgb, p)
        torch.cuda.synchronize()
        t1 = c.last_timings()
        assert t1["tuned"] == 1 and t1["workgroups"] >= 1
        assert (lab.cpu().numpy() == ref).all() and rep == ref_rep
    finally:
        c.close()
    c = gpu_lib.Context(0, timing=True, autotune=True, autotune_cache=cache)
    try:
        lab, rep = c.segment(rgb, p)
        torch.cuda.synchronize()
        t2 = c.last_timings()
        assert t2["tuned"] == 0 and t2["workgroups"] == t1["workgroups"]
        assert (lab.cpu().numpy() == ref).all()
    finally:
        c.close()


def _gate_helpers():
    from tests.test_gpu_gate import _dev, _he_case, _oracle_gated, _rand_model
    return _dev, _he_case, _oracle_gated, _rand_model


def test_coop_gated_matches_oracle(gpu_lib):
    """A gated single image on many workgroups: the levels before the gate
    and the gated levels in cooperative launches, the features and the
    network's bits in launches of their own between them.  Features, bits,
    labels and counters against the oracle, for the caller-supplied bits of
    rapid_segment too."""
    _dev, _he_case, _oracle_gated, _rand_model = _gate_helpers()
    img, p = _he_case()
    theta, wb = _rand_model(21)
    thresh, bits, ref, ref_rep, Xo = _oracle_gated(img, p, theta)
    for g, so in ((8, -1), (64, 4096)):
        with _shape(g, so):
            c = gpu_lib.Context(0, timing=True)
        try:
            _say("case: coop gated G=%d S=%d, marked %d of %d" % (g, so, bits.sum(), len(bits)))
            labs, reps, X, gb = c.segment_gated([_dev(img)], p, _dev(wb), thresh, features=True)
            assert c.last_timings()["workgroups"] == g
            assert np.abs(X.cpu().numpy() - Xo).max() <= 1e-6
            assert (gb.cpu().numpy() == bits).all()
            assert (labs[0].cpu().numpy() == ref).all()
            assert reps[0] == ref_rep
            lab, rep = c.segment(_dev(img), p, gate=_dev(bits))
            assert c.last_timings()["workgroups"] == g
            assert (lab.cpu().numpy() == ref).all() and rep == ref_rep
        finally:
            c.close()


@pytest.mark.parametrize("rule", ["either", "both", "differ"])
def test_coop_gated_nothing_marked(gpu_lib, rule):
    """No superpixel marked: no pair is active in the gated stages; labels
    and counters are the oracle's under an all-zero gate."""
    _dev, _he_case, _, _rand_model = _gate_helpers()
    img, p = _he_case()
    p = dict(p, gate_rule=rule)
    _, wb = _rand_model(21)
    K = oracle.n_superpixels(256, 192, p)
    ref, _, ref_rep = oracle.segment(img, p, gate=np.zeros(K, np.uint8))
    with _shape(16):
        c = gpu_lib.Context(0)
    try:
        _say("case: coop gated, nothing marked, rule %s" % rule)
        labs, reps, _, gb = c.segment_gated([_dev(img)], p, _dev(wb), 1e9)
        assert int(gb.sum().item()) == 0
        assert (labs[0].cpu().numpy() == ref).all()
        assert reps[0] == ref_rep
    finally:
        c.close()


def test_coop_gated_large_image(gpu_lib):
    """A 1024^2 H&E image with K = 4096, gated at the second level, spreads
    over a cooperative launch without being asked to (it is large; the
    autotuner picks the shape, and the gate point runs across the grid):
    labels and counters against the oracle under the GPU's bits, and
    features, bits and labels against the one-workgroup launch's."""
    _dev, _, _, _rand_model = _gate_helpers()
    img = synth.he_tile(1024, 1024, seed=33)
    p = params.default_params(1024, 1024, 4096, levels=params.THREE_LEVEL, gate_level=1)
    theta, wb = _rand_model(23)
    c = gpu_lib.Context(0, timing=True, autotune=True)
    try:
        _say("case: coop gated 1024^2 K=4096")
        labs, reps, X, gb = c.segment_gated([_dev(img)], p, _dev(wb), 0.0, features=True)
        t = c.last_timings()
        if t["workgroups"] > 1:
            assert t["pyramid"] == 1   # pyramid, levels and gate point: one launch
        gbits = gb.cpu().numpy()
        ref, _, ref_rep = oracle.segment(img, p, gate=gbits)
        assert (labs[0].cpu().numpy() == ref).all()
        assert reps[0] == ref_rep
    finally:
        c.close()
    # the single-launch route (one workgroup, gate inside the launch) for
    # the same image decides the same bits from the same features
    old = os.environ.get("RAPID_SHAPE")
    os.environ["RAPID_SHAPE"] = "1024,0,0"
    try:
        c = gpu_lib.Context(0)
    finally:
        if old is None:
            os.environ.pop("RAPID_SHAPE", None)
        else:
            os.environ["RAPID_SHAPE"] = old
    try:
        labs1, _, X1, gb1 = c.segment_gated([_dev(img)], p, _dev(wb), 0.0, features=True)
        assert (X1.cpu().numpy() == X.cpu().numpy()).all()
        assert (gb1.cpu().numpy() == gbits).all()
        assert (labs1[0].cpu().numpy() == labs[0].cpu().numpy()).all()
    finally:
        c.close()
    _say("autotuned shape of the gated levels: %d workgroups" % t["workgroups"])


def test_coop_he8192_max_size_matches_one_workgroup(gpu_lib):
    """The largest single image the boundary accepts (8192^2, K = 65536,
    three levels) on 64 workgroups with small sweeps on one workgroup, as
    the benchmark's autotuner picks it, equals the one-workgroup launch
    (whose parity with the oracle the 4096^2 and smaller cases pin) in
    labels, statistics-derived counters and every stage report."""
    import torch
    rgb = synth_gpu.he_slide(8192, 8192, seed=3, background=0.3, device="cuda")
    p = params.config3(8192, 8192, 65536)
    out = []
    for g, so in ((1, -1), (64, 16384)):
        with _shape(g, so):
            c = gpu_lib.Context(0, timing=True)
        try:
            _say("case: 8192^2 K=65536, G=%d S=%d" % (g, so))
            lab, rep = c.segment(rgb, p)
            torch.cuda.synchronize()
            assert c.last_timings()["workgroups"] == g
            out.append((lab, rep))
        finally:
            c.close()
    (l1, r1), (l2, r2) = out
    assert bool((l1 == l2).all().item())
    assert r1 == r2
    assert int(l2.min().item()) == 0 and int(l2.max().item()) == 65535


@pytest.mark.parametrize("max_sweeps", [1, 2, 5])
def test_coop_sweep_cap_unconverged_stages(gpu_lib, max_sweeps):
    """Sweep caps that end stages unconverged (the class counts then stand
    swapped at the next stage) on 8 workgroups, with small sweeps on the
    grid, on one workgroup, or all on one workgroup: labels and stage
    reports ("not converged" included) equal the oracle's."""
    img = synth.voronoi_gradient(481, 321, seed=1003)
    p = params.config2(481, 321)
    p["max_sweeps"] = max_sweeps
    ref, _, ref_rep = oracle.segment(img, p)
    assert any(not r["converged"] for r in ref_rep)
    for so in (-1, 2048, 1 << 30):
        with _shape(8, so):
            c = gpu_lib.Context(0)
        try:
            _say("case: coop G=8 S=%d max_sweeps %d" % (so, max_sweeps))
            got, rep = _run(c, img, p)
            assert (got == ref).all() and rep == ref_rep, (so, max_sweeps)
        finally:
            c.close()


def test_coop_abort_is_reported(gpu_lib, tmp_path):
    """A cooperative launch whose grid barrier gives up (forced from the host:
    the test hook raises the abort word before the launch, so every
    workgroup leaves at its first grid barrier) makes rapid_segment,
    rapid_refine_level and the gated route return RAPID_EDEVICE whether or
    not reports are asked for; a level-by-level state stays at its level;
    the autotuner drops the aborted candidates and keeps a one-workgroup
    shape, whose labels are the oracle's."""
    import torch
    img = synth.he_tile(256, 192, seed=71)
    p = params.default_params(256, 192, 48, levels=params.THREE_LEVEL)
    rgb = torch.from_numpy(img).cuda()
    with _shape(16, -1):
        c = gpu_lib.Context(0, timing=True, test_abort=True)
    try:
        for rep in (True, False):
            _say("case: forced abort, rapid_segment, report=%s" % rep)
            with pytest.raises(gpu_lib.RapidError) as e:
                c.segment(rgb, p, report=rep)
            assert e.value.code == -3
        _say("case: forced abort, level by level")
        st = c.state(rgb, p)
        with pytest.raises(gpu_lib.RapidError) as e:
            st.refine_level(0, report=False)
        assert e.value.code == -3
        # the state did not advance: level 1 is still out of order
        with pytest.raises(gpu_lib.RapidError) as e:
            st.refine_level(1, report=False)
        assert e.value.code == -4
        st.close()
    finally:
        c.close()
    # a gated large image on a cooperative launch (gate point across the grid)
    _dev, _, _, _rand_model = _gate_helpers()
    big = synth.he_tile(1024, 1024, seed=33)
    pg = params.default_params(1024, 1024, 4096, levels=params.THREE_LEVEL, gate_level=1)
    _, wb = _rand_model(23)
    with _shape(16, -1):
        c = gpu_lib.Context(0, test_abort=True)
    try:
        for rep in (True, False):
            _say("case: forced abort, gated large image, report=%s" % rep)
            with pytest.raises(gpu_lib.RapidError) as e:
                c.segment_gated([_dev(big)], pg, _dev(wb), 0.0, report=rep)
            assert e.value.code == -3
    finally:
        c.close()
    # the autotuner: every cooperative candidate aborts, a one-workgroup
    # shape is chosen and its labels are the oracle's
    ref, _, ref_rep = oracle.segment(img, p)
    cache = str(tmp_path / "tune.json")
    _say("case: forced abort, autotuner")
    c = gpu_lib.Context(0, timing=True, autotune=True, autotune_cache=cache, test_abort=True)
    try:
        lab, rep = c.segment(rgb, p)
        torch.cuda.synchronize()
        t = c.last_timings()
        assert t["tuned"] == 1 and t["workgroups"] == 1
        assert (lab.cpu().numpy() == ref).all() and rep == ref_rep
    finally:
        c.close()
    # and the same context without the hook runs the image cooperatively
    with _shape(16, -1):
        c = gpu_lib.Context(0, timing=True)
    try:
        _say("case: no abort after the forced ones")
        lab, rep = c.segment(rgb, p)
        torch.cuda.synchronize()
        assert c.last_timings()["workgroups"] == 16
        assert (lab.cpu().numpy() == ref).all() and rep == ref_rep
    finally:
        c.close()
