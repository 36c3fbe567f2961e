"""The sequential FIFO-queue baseline of the oracle (Algorithm RAPID's
boundary queue read literally), used to compare schedules with the
synchronous class sweeps.  Pins: the hand-worked step edges snap exactly
under it too; debug runs keep every invariant; it lowers Eq. (1) from the
grid and lands near the synchronous schedule's energy."""
import numpy as np
import pytest

import oracle
from paper_1704_02083_amd import params, synth
from tests.test_oracle_pins import _edge_params


def test_fifo_step_edges_snap():
    img = np.zeros((64, 64, 3), np.uint8)
    img[:, :37] = 50
    img[:, 37:] = 200
    lab, _, moves = oracle.segment_fifo(img, _edge_params(), debug=True)
    assert (lab == (np.mgrid[0:64, 0:64][1] >= 37)).all() and moves > 0
    img = np.zeros((64, 64, 3), np.uint8)
    img[27:] = 50
    img[:27] = 200
    lab, _, _ = oracle.segment_fifo(img, _edge_params(K=0, gx=1, gy=2), debug=True)
    assert (lab == (np.mgrid[0:64, 0:64][0] >= 27)).all()


@pytest.mark.parametrize("seed", range(4))
def test_fifo_invariants_and_energy(seed):
    W, H = 96 + 7 * seed, 64 + 5 * seed
    img = synth.voronoi_blur(W, H, regions=8, seed=seed)
    p = params.default_params(W, H, 12, levels=params.THREE_LEVEL if seed % 2 else [(1, [8, 4, 2, 1])])
    lab, st, moves = oracle.segment_fifo(img, p, debug=True)   # invariants checked per stage
    K = oracle.n_superpixels(W, H, p)
    assert (st[:, 0] > 0).all() and st[:, 0].sum() == W * H
    assert np.bincount(lab.ravel(), minlength=K).tolist() == st[:, 0].tolist()
    grid = oracle.init_labels(W, H, p["levels"][0][0] * p["levels"][0][1][0], *oracle.grid(W, H, 12))
    assert oracle.energy(img, p, lab) < oracle.energy(img, p, grid)


def test_fifo_energy_near_sync_schedule():
    """On BSD-shaped images both schedules cut Eq. (1) about tenfold from the
    grid and end within 20 % of each other (different local optima)."""
    for img in synth.batch_images(3):
        H, W = img.shape[:2]
        p = params.config2(W, H)
        lab_s, _, _ = oracle.segment(img, p)
        lab_f, _, _ = oracle.segment_fifo(img, p)
        es, ef = oracle.energy(img, p, lab_s), oracle.energy(img, p, lab_f)
        e0 = oracle.energy(img, p, oracle.init_labels(W, H, 16, *oracle.grid(W, H, 400)))
        assert es < e0 / 5 and ef < e0 / 5
        assert abs(ef - es) < 0.2 * es


def test_fifo_refuses_merge():
    img = synth.voronoi_blur(64, 64, regions=4, seed=1)
    p = dict(params.default_params(64, 64, 4), merge=True)
    with pytest.raises(RuntimeError):
        oracle.segment_fifo(img, p)
