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
