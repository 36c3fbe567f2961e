"""Host checks of the benchmark's algorithmic byte count (the roofline's
numerator): per stage one scan of the label map (4 B per block, skipped by a
gated stage that did nothing), 6 B per block visit, 4 + 96 B per commit,
3 B per pixel when the launch builds the pyramid, 4 B per output pixel; and
the profile summaries' traffic is used only for the kernel sources it was
taken on."""
import os

import numpy as np

import bench


def _rep(block, active, commits, sweeps):
    return {"block": block, "active": active, "commits": commits, "sweeps": sweeps}


def test_stage_bytes_by_hand():
    # 10 x 6 image: 15 blocks at B = 2, 60 at B = 1
    rep = [_rep(2, 7, 3, 2), _rep(1, 20, 5, 3)]
    want = 3 * 60 + (4 * 15 + 6 * 7 + 100 * 3) + (4 * 60 + 6 * 20 + 100 * 5)
    assert bench.stage_bytes(10, 6, rep, True) == want
    assert bench.stage_bytes(10, 6, rep, False) == want - 3 * 60
    # a gated stage that found nothing to do reads nothing
    assert bench.stage_bytes(10, 6, rep + [_rep(1, 0, 0, 0)], True) == want


def test_refine_alg_bytes_pyramid_rule():
    img = np.zeros((6, 10, 3), np.uint8)
    rep = [_rep(2, 7, 3, 2), _rep(1, 20, 5, 3)]
    stages = bench.stage_bytes(10, 6, rep, False)
    # one image: the pyramid comes from separate launches unless the launch says otherwise
    assert bench.refine_alg_bytes([img], [rep]) == 4 * 60 + stages
    assert bench.refine_alg_bytes([img], [rep], pyramid=True) == 4 * 60 + stages + 3 * 60
    # a batch of PYRAMID_MIN_JOBS images builds its pyramids in the launch
    n = bench.PYRAMID_MIN_JOBS
    assert bench.refine_alg_bytes([img] * n, [rep] * n) == n * (4 * 60 + stages + 3 * 60)


def test_profile_traffic_needs_matching_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k_refine_wl_counters.txt").write_text("k_refine:\n  source_hash: abc123\n  hbm_bytes_per_launch: 1.5e+09\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.profile_traffic("k_refine", "wl", "abc123") == 1.5e9
    assert bench.profile_traffic("k_refine", "wl", "def456") is None
    assert bench.profile_traffic("k_refine", "other", "abc123") is None
    assert os.path.exists(str(prof / "k_refine_wl_counters.txt"))
