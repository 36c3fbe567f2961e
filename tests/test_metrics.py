"""Pins of the agreement metrics (boundary recall, undersegmentation error)."""
import numpy as np

from paper_1704_02083_amd import metrics


def test_identical_maps():
    lab = np.random.default_rng(0).integers(0, 5, size=(20, 30))
    assert metrics.boundary_recall(lab, lab) == 1.0
    assert metrics.undersegmentation_error(lab, lab) == 0.0
    assert metrics.disagreement(lab, lab) == 0.0


def test_one_pixel_shift_of_a_straight_boundary():
    """Reference split at x = 10, test at x = 11 on a 40 x 16 image: every
    reference boundary pixel has a test boundary pixel one column away (BR
    = 1 at r = 2); the moved column costs H for each of the two reference
    segments (UE = 2H / (W H) = 2 / W); one column of W disagrees."""
    W, H = 40, 16
    xs = np.mgrid[0:H, 0:W][1]
    ref = (xs >= 10).astype(np.int32)
    test = (xs >= 11).astype(np.int32)
    assert metrics.boundary_recall(ref, test) == 1.0
    assert abs(metrics.undersegmentation_error(ref, test) - 2 / W) < 1e-12
    assert abs(metrics.disagreement(ref, test) - 1 / W) < 1e-12


def test_recall_radius():
    """A 3-px shift leaves the reference boundary columns 2 and 3 px away
    from the nearest test boundary: column 9 (3 px from column 12) is lost at
    r = 2, column 10 (2 px) is kept; at r = 3 both are kept."""
    W, H = 40, 8
    xs = np.mgrid[0:H, 0:W][1]
    ref = (xs >= 10).astype(np.int32)
    test = (xs >= 13).astype(np.int32)
    assert abs(metrics.boundary_recall(ref, test, r=2) - 0.5) < 1e-12
    assert metrics.boundary_recall(ref, test, r=3) == 1.0


def test_undersegmentation_of_a_merge():
    """A test segment spanning two reference halves of sizes a and b leaks
    min(a, b) pixels from each: UE = 2 min(a, b) / N."""
    ref = np.zeros((10, 10), np.int32)
    ref[:, 7:] = 1
    test = np.zeros((10, 10), np.int32)
    assert abs(metrics.undersegmentation_error(ref, test) - 2 * 30 / 100) < 1e-12


def test_roi_scores_by_hand():
    """Pixel precision/recall/F1 of a predicted ROI mask: 4 true positives,
    2 false positives, 1 false negative."""
    import torch
    from paper_1704_02083_amd import gate
    truth = torch.tensor([[1, 1, 1, 1, 1, 0, 0, 0]], dtype=torch.bool)
    pred = torch.tensor([[1, 1, 1, 1, 0, 1, 1, 0]], dtype=torch.bool)
    r = gate.roi_scores(pred, truth)
    assert abs(r["precision"] - 4 / 6) < 1e-12 and abs(r["recall"] - 4 / 5) < 1e-12
    assert abs(r["f1"] - 2 * (4 / 6) * (4 / 5) / (4 / 6 + 4 / 5)) < 1e-12


def test_roi_mask_maps_superpixel_classes():
    import torch
    from paper_1704_02083_amd import gate
    labels = torch.tensor([[0, 0, 1], [2, 1, 1]], dtype=torch.int32)
    g = torch.tensor([1, 0, 1], dtype=torch.uint8)
    assert gate.roi_mask(labels, g).tolist() == [[True, True, False], [True, False, False]]


def test_gate_model_round_trip(tmp_path):
    """A trained gate survives save/load bit for bit (no pickled objects)."""
    import torch
    from oracle import mlp
    from paper_1704_02083_amd import gate
    theta = gate.init_master(5)
    wb = torch.from_numpy(mlp.to_bf16_bits(theta).view(np.int16))
    path = str(tmp_path / "gate.npz")
    gate.save_model(path, torch.from_numpy(theta), wb, thresh=0.75, gate_level=3, rule="both")
    m, w, meta = gate.load_model(path, device="cpu")
    assert (m.numpy() == theta).all() and (w.numpy() == wb.numpy()).all()
    assert meta == {"thresh": 0.75, "gate_level": 3, "rule": "both"}
    np.savez(str(tmp_path / "bad.npz"), master=np.zeros(3, np.float32), w_bf16=np.zeros(3, np.int16),
             thresh=0.0, gate_level=3, rule=np.array("both"))
    import pytest
    with pytest.raises(ValueError):
        gate.load_model(str(tmp_path / "bad.npz"), device="cpu")
