"""Pins of the boundary-recall miss counts (the gate's training target)."""
import numpy as np

from oracle import targets
from paper_1704_02083_amd import metrics


def _halves(W, H, xb):
    lab = np.zeros((H, W), np.int32)
    lab[:, xb:] = 1
    return lab


def test_shifted_straight_boundary_by_hand():
    """Reference boundary between columns 31 | 32, test boundary between
    34 | 35: the reference boundary pixels sit in columns 31 and 32, the
    test ones in 34 and 35.  Column 32 is 2 away from column 34, column 31
    is 3 away."""
    ref, test = _halves(64, 40, 32), _halves(64, 40, 35)
    # (r, misses, charge to label 0, charge to label 1): column 31 is label 0
    # on both maps; column 32 is label 1 on the reference, 0 on the test
    for r, exp, c0, c1 in ((1, 80, 120, 40), (2, 40, 80, 0), (3, 0, 0, 0), (4, 0, 0, 0)):
        miss, nb, nm = targets.boundary_miss(ref, test, r, 2)
        assert nb == 80 and nm == exp, r
        assert miss[0] == c0 and miss[1] == c1, r


def test_identical_maps_have_no_misses():
    rng = np.random.default_rng(0)
    lab = rng.integers(0, 5, size=(23, 31)).astype(np.int32)
    miss, nb, nm = targets.boundary_miss(lab, lab, 0, 5)
    assert nm == 0 and miss.sum() == 0 and nb == targets.boundary_pixels(lab).sum()


def test_totals_agree_with_boundary_recall():
    """1 - misses / boundary pixels equals the boundary recall computed by
    dilation in the metrics module, on random blocky maps of ragged size."""
    rng = np.random.default_rng(1)
    for trial in range(6):
        H, W = int(rng.integers(9, 40)), int(rng.integers(9, 40))
        a = np.kron(rng.integers(0, 6, size=(8, 8)), np.ones((6, 6), np.int32))[:H, :W].astype(np.int32)
        b = np.kron(rng.integers(0, 6, size=(10, 10)), np.ones((4, 4), np.int32))[:H, :W].astype(np.int32)
        for r in (0, 1, 2, 4):
            _, nb, nm = targets.boundary_miss(a, b, r, 6)
            br = metrics.boundary_recall(a, b, r)
            assert abs((1 - nm / nb if nb else 1.0) - br) < 1e-12


def test_charge_goes_to_both_labels():
    """A missed pixel whose reference and test labels differ charges one
    to each."""
    ref = _halves(16, 4, 8)
    test = np.full((4, 16), 2, np.int32)   # no boundary at all in test
    miss, nb, nm = targets.boundary_miss(ref, test, 2, 3)
    assert nb == nm == 8
    assert list(miss) == [4, 4, 8]
