"""Parameter sets of the refinement sweep for the synthetic workloads.

The paper leaves the energy weights, size bounds and the level/stage
schedule unspecified (Eq. (1) and Algorithm RAPID name them but give no
values).  These are the defaults this project uses; all are integers.

  A          = floor(W H / K)              nominal superpixel area
  w_col      = A, w_pos = 100              SLIC-like compactness m = 10
  w_bnd      = 32 A                        one boundary edge = 32 colour^2 units
  frac_bits  = 4                           fixed-point fraction of the means
  min_size   = floor(A / 16) (or given)    hard lower bound on size
  max_size   = floor(3 A / 2)              the 1.5x upper size of Sec. 4.2
  max_sweeps = 64
"""
from __future__ import annotations

# single level, stages 16, 8, 4, 2, 1
SINGLE_LEVEL = [(1, [16, 8, 4, 2, 1])]
# three levels with linear ratio 4: effective block sizes 16 | 8, 4 | 2, 1
THREE_LEVEL = [(16, [1]), (4, [2, 1]), (1, [2, 1])]
# the same effective block sizes with the last level split in two (levels
# are exact box sums, so the plain result is identical): 16 | 8, 4 | 2 | 1.
# The gated workloads gate the last level, the single-pixel stage.
GATED_LEVELS = [(16, [1]), (4, [2, 1]), (2, [1]), (1, [1])]
GATE_LEVEL = 3


def default_params(W: int, H: int, K: int, levels=None, min_size: int | None = None,
                   gate_level: int = -1, max_sweeps: int = 64) -> dict:
    A = (W * H) // K
    return {
        "K": K, "gx": 0, "gy": 0,
        "levels": [(f, list(st)) for f, st in (levels or SINGLE_LEVEL)],
        "gate_level": gate_level,
        "frac_bits": 4,
        "max_sweeps": max_sweeps,
        "min_size": A // 16 if min_size is None else min_size,
        "max_size": (3 * A) // 2,
        "w_col": min(A, 4096),
        "w_pos": 100,
        "w_bnd": min(32 * A, 1 << 24),
    }


def config1() -> dict:
    """256x256, K = 64, min size 64 px, single level 16..1."""
    return default_params(256, 256, 64, min_size=64)


def config2(W: int, H: int) -> dict:
    """BSD500-shaped image, K = 400, single level 16..1."""
    return default_params(W, H, 400)


def config3(W: int = 4096, H: int = 4096, K: int = 16384, gate_level: int = -1) -> dict:
    """H&E tile, three levels of ratio 4."""
    return default_params(W, H, K, levels=THREE_LEVEL, gate_level=gate_level)


def gated(W: int, H: int, K: int, rule: str = "both", gate_level: int = GATE_LEVEL) -> dict:
    """H&E tile or slide tile under the learned gate: the schedule of
    config3 with the single-pixel stage as its own level; by default that
    last level is gated (gate_level 2 gates the 2-px stage too)."""
    p = default_params(W, H, K, levels=GATED_LEVELS, gate_level=gate_level)
    p["gate_rule"] = rule
    return p
