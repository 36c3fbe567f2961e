"""Slides: tiles with halos in one launch, core pixels written with
slide-wide superpixel ids; every tile equals an independent oracle run on
its core plus halo."""
import numpy as np
import pytest

import oracle
from paper_1704_02083_amd import params, rapid, synth_gpu

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0)
    yield c
    c.close()


def _tile_params(p_base, t):
    p = dict(p_base)
    p.update(K=0, gx=t["gx"], gy=t["gy"])
    return p


def _expected(img, p_base, lay, W, H):
    out = np.full((H, W), -1, np.int64)
    for t in lay:
        ex0, ey0, ex1, ey1 = t["ext"]
        cx0, cy0, cx1, cy1 = t["core"]
        sub = np.ascontiguousarray(img[ey0:ey1, ex0:ex1])
        lab, _, _ = oracle.segment(sub, _tile_params(p_base, t))
        gid = (t["gid_y0"] + lab // t["gx"]) * t["gid_w"] + t["gid_x0"] + lab % t["gx"]
        out[cy0:cy1, cx0:cx1] = gid[cy0 - ey0:cy1 - ey0, cx0 - ex0:cx1 - ex0]
    return out


@pytest.mark.parametrize("W,H,tile,halo", [(1000, 700, 256, 64), (640, 512, 320, 32)])
def test_slide_matches_tilewise_oracle(ctx, W, H, tile, halo):
    import torch
    _say("case: slide %dx%d tile %d halo %d" % (W, H, tile, halo))
    rgb = synth_gpu.he_slide(W, H, seed=4, device="cuda", band=256)
    p = params.default_params(W, H, 1, levels=params.THREE_LEVEL)
    p["min_size"], p["max_size"], p["w_col"], p["w_bnd"] = 64, 1536, 1024, 32 * 1024
    labels, _ = ctx.segment_slide(rgb, p, tile=tile, halo=halo, cell=32)
    torch.cuda.synchronize()
    img = rgb.cpu().numpy()
    lay = rapid.tile_layout(W, H, tile, halo, 32)
    exp = _expected(img, p, lay, W, H)
    got = labels.cpu().numpy()
    assert (exp >= 0).all()
    mism = int((got != exp).sum())
    assert mism == 0, "%d slide labels differ" % mism


@pytest.mark.parametrize("wgs", [1, 3, 5])
def test_persistent_queue_few_workgroups(gpu_lib, wgs):
    """The refinement launch as a persistent kernel over its job queue with
    fewer workgroups than tiles (RAPID_SHAPE's sixth field): each workgroup
    refines tile after tile, largest first, and every tile still equals its
    oracle run."""
    import os
    import torch
    W, H, T, h = 1000, 700, 256, 64
    old = os.environ.get("RAPID_SHAPE")
    os.environ["RAPID_SHAPE"] = "1024,0,1,1,-1,%d" % wgs
    try:
        c = gpu_lib.Context(0, timing=True)
    finally:
        if old is None:
            os.environ.pop("RAPID_SHAPE", None)
        else:
            os.environ["RAPID_SHAPE"] = old
    try:
        _say("case: slide %dx%d on %d persistent workgroups" % (W, H, wgs))
        rgb = synth_gpu.he_slide(W, H, seed=4, device="cuda", band=256)
        p = params.default_params(W, H, 1, levels=params.THREE_LEVEL)
        p["min_size"], p["max_size"], p["w_col"], p["w_bnd"] = 64, 1536, 1024, 32 * 1024
        labels, reps = c.segment_slide(rgb, p, tile=T, halo=h, cell=32, report=True)
        torch.cuda.synchronize()
        lay = rapid.tile_layout(W, H, T, h, 32)
        exp = _expected(rgb.cpu().numpy(), p, lay, W, H)
        assert (labels.cpu().numpy() == exp).all()
        # the reports stay in tile order whatever order the queue ran them in
        for t, rp in zip(lay, reps):
            ex0, ey0, ex1, ey1 = t["ext"]
            sub = np.ascontiguousarray(rgb[ey0:ey1, ex0:ex1].cpu().numpy())
            _, _, ref_rep = oracle.segment(sub, _tile_params(p, t))
            assert rp == ref_rep
    finally:
        c.close()
