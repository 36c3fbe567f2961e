"""The seeded input generators (no method arithmetic): determinism, shapes,
value ranges and the structure the workloads specify -- background fraction,
tissue colours, nucleus density, seamless row bands."""
import numpy as np
import pytest
import torch

from paper_1704_02083_amd import synth, synth_gpu


def test_voronoi_blur_deterministic_and_in_range():
    a, b = synth.voronoi_blur(), synth.voronoi_blur()
    assert a.shape == (256, 256, 3) and a.dtype == np.uint8
    assert (a == b).all()
    assert not (a == synth.voronoi_blur(seed=2)).all()
    # 24 regions of uniform random colour: many distinct colours, full range
    assert a.min() < 40 and a.max() > 215


def test_batch_shapes_and_seeds():
    imgs = synth.batch_images(6)
    assert [im.shape for im in imgs] == [(321, 481, 3)] * 3 + [(481, 321, 3)] * 3
    again = synth.batch_images(6)
    assert all((x == y).all() for x, y in zip(imgs, again))
    assert not (imgs[0] == imgs[1]).all()


def test_he_tile_background_and_nuclei():
    img = synth.he_tile(512, 512, seed=3, background=0.30)
    grey = (img[..., 0] == img[..., 1]) & (img[..., 1] == img[..., 2]) & (img[..., 0] >= 230)
    assert abs(grey.mean() - 0.30) < 0.02
    tissue = ~grey
    dark = tissue & (img[..., 0] < 130) & (img[..., 2] > img[..., 1])   # purple nuclei
    # one nucleus (mean area ~ pi 5.5^2 ~ 95 px) per 400 px^2 of tissue
    frac = dark.sum() / tissue.sum()
    assert 0.08 < frac < 0.35, frac


def test_he_slide_bands_are_seamless_and_deterministic():
    a = synth_gpu.he_slide(320, 200, seed=9, background=0.4, device="cpu", band=64)
    b = synth_gpu.he_slide(320, 200, seed=9, background=0.4, device="cpu", band=1024)
    assert a.shape == (200, 320, 3) and a.dtype == torch.uint8
    assert torch.equal(a, b)
    c = synth_gpu.he_slide(320, 200, seed=10, background=0.4, device="cpu")
    assert not torch.equal(a, c)


def test_he_slide_structure():
    W = H = 768
    img = synth_gpu.he_slide(W, H, seed=4, background=0.4, device="cpu").numpy()
    mask = synth_gpu.tissue_mask(W, H, seed=4, background=0.4, device="cpu").numpy()
    # the background quantile is taken on a 16-px subsample of the mask
    assert abs((~mask).mean() - 0.4) < 0.03
    bg = img[~mask]
    assert (bg[:, 0] == bg[:, 1]).all() and (bg[:, 1] == bg[:, 2]).all()
    assert bg.min() >= 230 and bg.max() <= 245
    t = img[mask].astype(np.int32)
    nuc = (t[:, 0] < 130) & (t[:, 2] > t[:, 1])
    assert 0.08 < nuc.mean() < 0.35, nuc.mean()
    # the rest of the tissue lies between the lilac base and the stroma colour, +-15
    rest = t[~nuc]
    assert rest[:, 0].min() >= 200 - 15 - 1 and rest[:, 0].max() <= 220 + 15 + 1
    assert rest[:, 1].min() >= 150 - 15 - 1 and rest[:, 1].max() <= 160 + 15 + 1


@pytest.mark.gpu
def test_he_slide_gpu_matches_cpu():
    """The same counter-based hashes on the GPU: identical images up to a
    rare one-step rounding difference of the float noise."""
    a = synth_gpu.he_slide(512, 256, seed=7, device="cpu")
    b = synth_gpu.he_slide(512, 256, seed=7, device="cuda").cpu()
    d = (a.int() - b.int()).abs()
    assert d.max() <= 1 and (d == 0).float().mean() > 0.999
