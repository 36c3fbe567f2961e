"""Randomised parity sweep: seeded random image sizes, schedules, weights,
size bounds, fixed-point bits, sweep caps, merge on or off, gates with random
rules and bits, and random launch shapes (workgroup size, residency, pyramid
placement): labels, statistics counters and stage reports bit-exact against
the oracle in every case."""
import os

import numpy as np
import pytest

import oracle
from paper_1704_02083_amd import params, synth

pytestmark = pytest.mark.gpu

SCHEDULES = [
    [(1, [16, 8, 4, 2, 1])],
    [(1, [8, 4, 2, 1])],
    [(1, [4, 2, 1])],
    [(4, [2, 1]), (1, [2, 1])],
    [(16, [1]), (4, [2, 1]), (1, [2, 1])],
    [(8, [1]), (2, [2, 1]), (1, [1])],
    [(1, [32, 16, 8, 4, 2, 1])],
]


def _case(seed, large=False):
    rng = np.random.default_rng(1000 + seed)
    for _ in range(50):
        lo, hi = (400, 1200) if large else (20, 220)
        W, H = int(rng.integers(lo, hi)), int(rng.integers(lo, hi))
        levels = SCHEDULES[int(rng.integers(len(SCHEDULES)))]
        K = int(rng.integers(200, 3000)) if large else int(rng.integers(1, 60))
        p = params.default_params(W, H, K, levels=levels)
        p.update(w_col=int(rng.integers(0, 5000)), w_pos=int(rng.integers(0, 400)),
                 w_bnd=int(rng.integers(0, 1 << 18)), frac_bits=int(rng.integers(0, 5)),
                 max_sweeps=int(rng.integers(1, 48)), merge=bool(rng.random() < 0.4))
        A = max(1, (W * H) // max(1, K))
        p["min_size"] = int(rng.integers(0, max(1, A // 2)))
        p["max_size"] = int(rng.integers(max(2, A), 3 * A + 2))
        if len(levels) > 1 and rng.random() < 0.5:
            p["gate_level"] = int(rng.integers(1, len(levels)))
            p["gate_rule"] = ["either", "both", "differ"][int(rng.integers(3))]
        try:
            oracle.n_superpixels(W, H, p)
            img = synth.voronoi_gradient(W, H, seed=seed, regions=(3, 20))
            oracle.segment(img, p)   # refuses infeasible grids and parameters
        except (RuntimeError, ValueError):
            continue
        return rng, W, H, p, img
    pytest.skip("no feasible case drawn")


@pytest.mark.parametrize("seed,large", [(s, False) for s in range(64)] + [(100 + s, True) for s in range(8)])
def test_random_configuration(gpu_lib, seed, large):
    """Small images in 64 cases; 8 cases of 400-1200 px with up to 3000
    superpixels, where the per-superpixel state outgrows LDS and classes
    take several passes of the workgroup."""
    import torch
    rng = np.random.default_rng(5000 + seed)
    _, W, H, p, img = _case(seed, large)
    Kp = oracle.n_superpixels(W, H, p)
    gate = (rng.random(Kp) < 0.5).astype(np.uint8) if p["gate_level"] >= 0 else None
    ref, ref_stats, ref_rep = oracle.segment(img, p, gate=gate)
    shape = "%d,%d,%d" % (int(rng.choice([256, 512, 1024])), int(rng.integers(0, 4)), int(rng.integers(0, 2)))
    old = os.environ.get("RAPID_SHAPE")
    os.environ["RAPID_SHAPE"] = shape
    try:
        print("case: seed %d %dx%d K'=%d levels %s merge %s gate %s shape %s" % (
            seed, W, H, Kp, p["levels"], p["merge"], p.get("gate_rule") if gate is not None else None, shape),
            flush=True)
        c = gpu_lib.Context(0)
        g = None if gate is None else torch.from_numpy(gate).cuda()
        lab, rep = c.segment(torch.from_numpy(img).cuda(), p, gate=g)
        torch.cuda.synchronize()
        assert (lab.cpu().numpy() == ref).all()
        assert rep == ref_rep
        c.close()
    finally:
        if old is None:
            os.environ.pop("RAPID_SHAPE", None)
        else:
            os.environ["RAPID_SHAPE"] = old


@pytest.mark.parametrize("seed,large", [(s, False) for s in range(64)] + [(100 + s, True) for s in range(8)])
def test_random_configuration_cooperative(gpu_lib, seed, large):
    """The same 72 cases with the image spread over a cooperative launch of
    random size, small sweeps on one workgroup at a random threshold (never,
    some, every sweep): sweep caps that end stages unconverged, caller gate
    bits and every schedule against the oracle (merge cases fall back to one
    workgroup and must still match)."""
    import torch
    rng = np.random.default_rng(7000 + seed)
    _, W, H, p, img = _case(seed, large)
    Kp = oracle.n_superpixels(W, H, p)
    gate = (rng.random(Kp) < 0.5).astype(np.uint8) if p["gate_level"] >= 0 else None
    ref, ref_stats, ref_rep = oracle.segment(img, p, gate=gate)
    groups = int(rng.choice([2, 4, 8, 32, 64]))
    solo = int(rng.choice([-1, 64, 1024, 1 << 30]))
    shape = "1024,0,0,%d,%d" % (groups, solo)
    old = os.environ.get("RAPID_SHAPE")
    os.environ["RAPID_SHAPE"] = shape
    try:
        print("case: seed %d %dx%d K'=%d levels %s sweeps %d merge %s gate %s shape %s" % (
            seed, W, H, Kp, p["levels"], p["max_sweeps"], p["merge"],
            p.get("gate_rule") if gate is not None else None, shape), flush=True)
        c = gpu_lib.Context(0, timing=True)
        g = None if gate is None else torch.from_numpy(gate).cuda()
        lab, rep = c.segment(torch.from_numpy(img).cuda(), p, gate=g)
        torch.cuda.synchronize()
        assert c.last_timings()["workgroups"] == (1 if p["merge"] else groups)
        assert (lab.cpu().numpy() == ref).all()
        assert rep == ref_rep
        c.close()
    finally:
        if old is None:
            os.environ.pop("RAPID_SHAPE", None)
        else:
            os.environ["RAPID_SHAPE"] = old


def _fused_case(seed):
    """A random H&E crop, grid, schedule, gate level and rule for the fused
    gate (the network decides the bits inside the refinement launch)."""
    rng = np.random.default_rng(777 + seed)
    for _ in range(50):
        W, H = int(rng.integers(200, 1100)), int(rng.integers(200, 900))
        K = int(rng.integers(48, 3500))
        levels = [params.THREE_LEVEL, params.GATED_LEVELS][int(rng.integers(2))]
        p = params.default_params(W, H, K, levels=levels, gate_level=int(rng.integers(1, len(levels))))
        p["gate_rule"] = ["either", "both", "differ"][int(rng.integers(3))]
        img = synth.he_tile(W, H, seed=900 + seed)
        try:
            oracle.segment(img, dict(p, gate_level=-1))   # refuses infeasible grids and parameters
        except (RuntimeError, ValueError):
            continue
        return rng, W, H, p, img
    pytest.skip("no feasible case drawn")


@pytest.mark.parametrize("seed", range(16))
def test_random_fused_gate(gpu_lib, seed):
    """The fused gate on random H&E crops: a random network (He init, bf16),
    its threshold at a random quantile of its logits, a random launch shape
    (workgroup size, residency, pyramid placement); labels and stage reports
    against the oracle run under the GPU's own gate bits."""
    import torch
    from oracle import mlp
    rng, W, H, p, img = _fused_case(seed)
    theta = mlp.he_init(int(rng.integers(1000))).astype(np.float32)
    wb = torch.from_numpy(mlp.to_bf16_bits(theta).view(np.int16)).cuda()
    shape = "%d,%d,%d" % (int(rng.choice([256, 512, 1024])), int(rng.integers(0, 4)), int(rng.integers(0, 2)))
    old = os.environ.get("RAPID_SHAPE")
    os.environ["RAPID_SHAPE"] = shape
    try:
        c = gpu_lib.Context(0)
    finally:
        if old is None:
            os.environ.pop("RAPID_SHAPE", None)
        else:
            os.environ["RAPID_SHAPE"] = old
    try:
        rgb = torch.from_numpy(img).cuda()
        _, _, X, _ = c.segment_gated([rgb], p, wb, 1e9, features=True, report=False)
        z, _ = mlp.forward(theta.astype(np.float64), X.cpu().numpy().astype(np.float64), bf16=True)
        thresh = float(np.quantile(z, rng.uniform(0.2, 0.8)))
        print("case: fused seed %d %dx%d levels %d gate level %d rule %s shape %s" % (
            seed, W, H, len(p["levels"]), p["gate_level"], p["gate_rule"], shape), flush=True)
        labs, reps, _, g = c.segment_gated([rgb], p, wb, thresh)
        torch.cuda.synchronize()
        gb = g.cpu().numpy()
        ref, _, ref_rep = oracle.segment(img, p, gate=gb)
        assert (labs[0].cpu().numpy() == ref).all()
        assert reps[0] == ref_rep
    finally:
        c.close()
