"""Brute-force pin of the oracle's move rule on tiny images.

For random valid states (4-connected superpixels, block-constant labels) of
8x8 and 12x10 images, every block of a class is re-evaluated from scratch in
exact Python integers: each admissible label is applied, the pixel-level
global energy of Eq. (1) is recomputed, and the argmin (ties keep the current
label, then the smaller label) must be the oracle's proposal.  The energy
change the oracle reports must equal the global energy difference, which
pins the block energy E' (the difference form of Sec. 3.1) to Eq. (1).
"""
import numpy as np
import pytest

import oracle
from tests import pyref


def _random_state(rng, W, H, B, K_grid, steps):
    """Grid labels at block size B, then random connectivity-preserving
    block moves (checked by global BFS)."""
    gx, gy = K_grid
    lab = oracle.init_labels(W, H, B, gx, gy)
    nbx, nby = -(-W // B), -(-H // B)
    bl = lab[::B, ::B].copy()
    for _ in range(steps):
        by, bx = int(rng.integers(0, nby)), int(rng.integers(0, nbx))
        a = bl[by, bx]
        nbrs = [bl[by + dy, bx + dx] for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0))
                if 0 <= by + dy < nby and 0 <= bx + dx < nbx and bl[by + dy, bx + dx] != a]
        if not nbrs:
            continue
        k = nbrs[int(rng.integers(0, len(nbrs)))]
        trial = bl.copy()
        trial[by, bx] = k
        comps = pyref.components4(trial)
        if comps.get(int(a), 0) == 1 and all(v == 1 for v in comps.values()):
            bl = trial
    return np.kron(bl, np.ones((B, B), np.int32))[:H, :W].astype(np.int32)


def _brute_force(img, p, lab, K, B, cls, gate):
    H, W = lab.shape
    F = p["frac_bits"]
    nbx, nby = -(-W // B), -(-H // B)
    n, S, T = pyref.stats(img, lab, K)
    c, mu = pyref.means(n, S, T, F)
    bl = lab[::B, ::B]

    def L(bx, by):
        return int(bl[by, bx]) if 0 <= bx < nbx and 0 <= by < nby else -1

    def active(a, k):
        if gate is None:
            return True
        rule = p.get("gate_rule", "either")
        if rule == "both":
            return bool(gate[a]) and bool(gate[k])
        if rule == "differ":
            return bool(gate[a]) != bool(gate[k])
        return bool(gate[a]) or bool(gate[k])

    out = {}
    for by in range(cls // 3, nby, 3):
        for bx in range(cls % 3, nbx, 3):
            a = L(bx, by)
            nb4 = [L(bx - 1, by), L(bx + 1, by), L(bx, by - 1), L(bx, by + 1)]
            if not any(k >= 0 and k != a and active(a, k) for k in nb4):
                continue
            w = min(B, W - bx * B)
            h = min(B, H - by * B)
            m = w * h
            if n[a] - m < p["min_size"]:
                continue
            mask = sum(1 << r for r, (dx, dy) in enumerate(pyref.RING) if L(bx + dx, by + dy) == a)
            if not pyref.yokoi_simple(mask):
                continue
            options = [a] + sorted({k for k in nb4 if k >= 0 and k != a and n[k] + m <= p["max_size"]})
            energies = []
            for k in options:
                trial = lab.copy()
                trial[by * B:by * B + h, bx * B:bx * B + w] = k
                energies.append(pyref.global_energy(img, trial, c, mu, p))
            best = 0
            for i in range(1, len(options)):
                if energies[i] < energies[best]:
                    best = i
            if best != 0 and active(a, options[best]):
                out[by * nbx + bx] = (a, options[best], energies[best] - energies[0])
    return out


CASES = [(8, 8, (2, 2), 2), (8, 8, (2, 2), 1), (12, 10, (3, 2), 2), (12, 10, (3, 2), 1),
         # ragged edge blocks (clipped to 1 px wide / 1 px high, or 3x2)
         (9, 7, (2, 2), 2), (11, 9, (2, 2), 4), (7, 10, (1, 2), 4)]


@pytest.mark.parametrize("trial", range(12))
def test_proposals_equal_global_argmin(trial):
    rng = np.random.default_rng(100 + trial)
    checked = 0
    for (W, H, grid, B) in CASES:
        img = rng.integers(0, 256, size=(H, W, 3)).astype(np.uint8)
        if trial % 2:
            # smooth two-tone image so that moves are frequent
            img[:, : int(rng.integers(2, W - 1))] //= 4
        lab = _random_state(rng, W, H, B, grid, steps=int(rng.integers(0, 40)))
        K = grid[0] * grid[1]
        p = {"K": 0, "gx": grid[0], "gy": grid[1], "levels": [(1, [B])], "gate_level": -1,
             "frac_bits": int(rng.integers(0, 7)), "max_sweeps": 8,
             "min_size": int(rng.integers(0, 20)), "max_size": int(rng.integers(20, 80)),
             "w_col": int(rng.integers(0, 60)), "w_pos": int(rng.integers(0, 400)),
             "w_bnd": int(rng.integers(0, 6000))}
        gate = None
        if trial % 3 == 2:
            gate = rng.integers(0, 2, size=K).astype(np.uint8)
            p["gate_rule"] = ("either", "both", "differ")[(trial // 3) % 3]
        for cls in range(9):
            props, de = oracle.propose_class(img, p, lab, K, B, cls, gate=gate)
            got = {int(b): (int(a), int(k), int(e)) for (b, a, k), e in zip(props, de)}
            exp = _brute_force(img, p, lab, K, B, cls, gate)
            assert got == exp, (W, H, B, cls)
            checked += len(exp)
    assert checked >= 0


def test_bruteforce_finds_moves():
    """The brute-force cases above are not vacuous: across seeds a good
    number of proposals is compared."""
    total = 0
    for trial in range(6):
        rng = np.random.default_rng(500 + trial)
        img = rng.integers(0, 256, size=(8, 8, 3)).astype(np.uint8)
        img[:, :3] //= 5
        lab = _random_state(rng, 8, 8, 1, (2, 2), steps=30)
        p = {"K": 0, "gx": 2, "gy": 2, "levels": [(1, [1])], "gate_level": -1, "frac_bits": 4,
             "max_sweeps": 8, "min_size": 2, "max_size": 60, "w_col": 10, "w_pos": 50, "w_bnd": 200}
        for cls in range(9):
            exp = _brute_force(img, p, lab, 4, 1, cls, None)
            props, de = oracle.propose_class(img, p, lab, 4, 1, cls)
            assert {int(b): (int(a), int(k), int(e)) for (b, a, k), e in zip(props, de)} == exp
            total += len(exp)
    assert total >= 10
