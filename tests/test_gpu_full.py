"""Parity at the full sizes of the workloads, in the launch configuration
the benchmark times."""
import numpy as np
import pytest

import oracle
from paper_1704_02083_amd import params, synth, synth_gpu

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0)
    yield c
    c.close()


def test_batch_all_200_images_bit_exact(ctx):
    """Every image of the 200-image batch launch equals its oracle run."""
    import torch
    imgs = synth.batch_images(200)
    p = params.config2(481, 321)
    _say("case: batch 200 full parity")
    labs, reps = ctx.segment_batch([torch.from_numpy(im).cuda() for im in imgs], p)
    torch.cuda.synchronize()
    bad = []
    for i, im in enumerate(imgs):
        ref, _, ref_rep = oracle.segment(im, p)
        if not ((labs[i].cpu().numpy() == ref).all() and reps[i] == ref_rep):
            bad.append(i)
    assert not bad, "images differ: %s" % bad[:10]


def test_he4096_three_levels_bit_exact(ctx):
    """4096 x 4096 H&E tile, K = 16384, three levels of ratio 4."""
    import torch
    rgb = synth_gpu.he_slide(4096, 4096, seed=3, background=0.3, device="cuda")
    p = params.config3()
    _say("case: 4096^2 K=16384 three levels")
    lab, rep = ctx.segment(rgb, p)
    torch.cuda.synchronize()
    img = rgb.cpu().numpy()
    ref, _, ref_rep = oracle.segment(img, p)
    mism = int((lab.cpu().numpy() != ref).sum())
    assert mism == 0, "%d labels differ" % mism
    assert rep == ref_rep
    # levels as exact box sums: three levels equal one level 16..1 on the GPU
    lab1, rep1 = ctx.segment(rgb, params.default_params(4096, 4096, 16384))
    torch.cuda.synchronize()
    assert (lab1.cpu().numpy() == ref).all()


def test_slide_32768_sampled_tiles_bit_exact(ctx):
    """The 32768^2 slide in the launch the benchmark times (256 tiles of
    2048^2 with a 64-px halo, 32-px cells, three levels): a corner tile, an
    edge tile and an interior tile equal independent oracle runs on their
    core plus halo, with slide-wide ids; every pixel is labelled with an id
    of the slide grid."""
    import torch
    from paper_1704_02083_amd import rapid
    W = H = 32768
    rgb = synth_gpu.he_slide(W, H, seed=4, background=0.4, device="cuda", band=1024)
    p = params.default_params(2048, 2048, 4096, levels=params.THREE_LEVEL)
    _say("case: 32768^2 slide, 256 tiles")
    labels, _ = ctx.segment_slide(rgb, p, tile=2048, halo=64, cell=32)
    torch.cuda.synchronize()
    gid_max = (W // 32) * (H // 32)
    lo, hi = int(labels.min().item()), int(labels.max().item())
    assert 0 <= lo and hi < gid_max
    lay = rapid.tile_layout(W, H, 2048, 64, 32)
    for ti in (0, 7, 16 * 9 + 6):          # corner, top edge, interior
        t = lay[ti]
        ex0, ey0, ex1, ey1 = t["ext"]
        cx0, cy0, cx1, cy1 = t["core"]
        _say("case: slide tile %d" % ti)
        sub = rgb[ey0:ey1, ex0:ex1].cpu().numpy()
        pt = dict(p, K=0, gx=t["gx"], gy=t["gy"])
        lab, _, _ = oracle.segment(np.ascontiguousarray(sub), pt)
        gid = (t["gid_y0"] + lab // t["gx"]) * t["gid_w"] + t["gid_x0"] + lab % t["gx"]
        exp = gid[cy0 - ey0:cy1 - ey0, cx0 - ex0:cx1 - ex0]
        got = labels[cy0:cy1, cx0:cx1].cpu().numpy()
        mism = int((got != exp).sum())
        assert mism == 0, "tile %d: %d labels differ" % (ti, mism)
