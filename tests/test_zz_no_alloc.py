"""rapid_segment_noalloc, the allocation-free variant of rapid_segment for
callers that cannot allocate device memory: through the C-ABI, calls in a
row (the second with a smaller input, then a three-level image, caller gate
bits and a strided label buffer) give the labels and stage reports of
rapid_segment bit for bit, and of the oracle; an image whose scratch would
not fit the fixed device array is refused without queueing anything."""
import numpy as np
import pytest

import oracle
from paper_1704_02083_amd import params, synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def test_noalloc_matches_segment(gpu_lib):
    import torch
    c = gpu_lib.Context(0, timing=True)
    try:
        img_he = synth.he_tile(384, 256, seed=81)
        p_he = params.default_params(384, 256, 96, levels=params.THREE_LEVEL, gate_level=1)
        K_he = oracle.n_superpixels(384, 256, p_he)
        bits = (np.random.default_rng(81).random(K_he) < 0.4).astype(np.uint8)
        cases = [
            # the batched workload's shape, then a smaller image
            ("481x321 K=400", synth.voronoi_gradient(481, 321, seed=1003), params.config2(481, 321), None),
            ("200x150 K=30", synth.voronoi_blur(200, 150, regions=12, seed=77),
             params.default_params(200, 150, 30, min_size=30), None),
            ("384x256 three levels, gate bits", img_he, p_he, bits),
        ]
        # the existing entry point first, for every case
        want = []
        for name, img, p, g in cases:
            rgb = torch.from_numpy(img).cuda()
            gd = None if g is None else torch.from_numpy(g).cuda()
            lab, rep = c.segment(rgb, p, gate=gd)
            torch.cuda.synchronize()
            want.append((lab.cpu().numpy(), rep))
        # then the allocation-free one, calls back to back into
        # caller-allocated label buffers
        for (name, img, p, g), (lab_w, rep_w) in zip(cases, want):
            _say("case: noalloc %s" % name)
            rgb = torch.from_numpy(img).cuda()
            gd = None if g is None else torch.from_numpy(g).cuda()
            out = torch.full(img.shape[:2], -7, dtype=torch.int32, device="cuda")
            _, rep = c.segment_noalloc(rgb, p, gate=gd, labels=out)
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            assert (got == lab_w).all(), "%s: %d labels differ" % (name, int((got != lab_w).sum()))
            assert rep == rep_w
            ref, _, ref_rep = oracle.segment(img, p, gate=g)
            assert (got == ref).all() and rep == ref_rep
            assert c.last_timings()["workgroups"] == 1
        # a label buffer with a row stride wider than the image (the final
        # map is then written by the output phase, not in place)
        name, img, p, _ = cases[1]
        _say("case: noalloc strided labels")
        rgb = torch.from_numpy(img).cuda()
        wide = torch.full((img.shape[0], img.shape[1] + 24), -7, dtype=torch.int32, device="cuda")
        view = wide[:, :img.shape[1]]
        c.segment_noalloc(rgb, p, labels=view, report=False)
        torch.cuda.synchronize()
        assert (view.cpu().numpy() == want[1][0]).all()
        assert (wide[:, img.shape[1]:] == -7).all()
        # too large for the fixed array: refused, nothing written
        _say("case: noalloc too large")
        big = torch.zeros((2048, 2048, 3), dtype=torch.uint8, device="cuda")
        out = torch.full((2048, 2048), -7, dtype=torch.int32, device="cuda")
        with pytest.raises(gpu_lib.RapidError) as e:
            c.segment_noalloc(big, params.default_params(2048, 2048, 4096), labels=out)
        assert e.value.code == -1
        torch.cuda.synchronize()
        assert (out == -7).all()
    finally:
        c.close()


def test_noalloc_replays_from_a_hip_graph(gpu_lib):
    """rapid_segment_noalloc without a report queues kernels only (no
    allocation, no memset node, no synchronisation), so a caller can capture
    it in a HIP graph: captured once, the graph replays on new images copied
    into the captured input between replays (eager work and synchronisation
    in between), and every replay gives the labels of an eager call and of
    the oracle."""
    import torch
    s = torch.cuda.Stream()
    c = gpu_lib.Context(0, stream=s)
    try:
        W, H, K = 256, 192, 48
        p = params.default_params(W, H, K, levels=params.THREE_LEVEL)
        imgs = [synth.voronoi_blur(W, H, regions=14, seed=900 + i) for i in range(4)]
        rgb = torch.from_numpy(imgs[0]).cuda()
        out = torch.full((H, W), -7, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        # an eager call first loads the kernels and sets their LDS limits
        with torch.cuda.stream(s):
            c.segment_noalloc(rgb, p, labels=out, report=False)
        s.synchronize()
        g = torch.cuda.CUDAGraph()
        _say("case: noalloc graph capture %dx%d K=%d" % (W, H, K))
        with torch.cuda.graph(g, stream=s):
            c.segment_noalloc(rgb, p, labels=out, report=False)
        for i in (1, 2, 0, 3):
            _say("case: noalloc graph replay, image %d" % i)
            rgb.copy_(torch.from_numpy(imgs[i]))
            out.fill_(-7)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            eager = torch.full((H, W), -5, dtype=torch.int32, device="cuda")
            with torch.cuda.stream(s):
                c.segment(rgb, p, labels=eager, report=False)
            s.synchronize()
            assert (got == eager.cpu().numpy()).all(), "replay %d differs from the eager call" % i
            ref, _, _ = oracle.segment(imgs[i], p)
            assert (got == ref).all(), "replay %d differs from the oracle" % i
        del g
    finally:
        c.close()
