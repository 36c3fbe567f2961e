"""ctypes front of the plain CPU oracle (``oracle/rapid_oracle.c``).

Test infrastructure only: the tests, the smoke check and the benchmark's CPU
baseline use it; the product path never imports it.  It shares no code with
the GPU library; the only thing both sides consume is the seeded synthetic
image and the parameter dictionary built by the caller.

Parameter dictionary (also accepted by the GPU binding):
    K            target superpixel count (0: use gx, gy)
    gx, gy       explicit grid when K == 0
    levels       list of (factor, [block sizes in level pixels]) coarse→fine
    gate_level   first level refined under the gate (-1: never)
    gate_rule    "either" (default), "both" or "differ": the pairs a gate lets
                 move
    frac_bits    fixed-point fraction bits F of the means
    max_sweeps   sweep cap per stage
    min_size, max_size   hard size bounds in pixels
    w_col, w_pos, w_bnd  integer energy weights
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rapid_oracle.c")
_LIB = os.path.join(_HERE, "librapid_oracle.so")

MAX_LEVELS = 4
GATE_RULES = {"either": 0, "both": 1, "differ": 2}
MAX_STAGES = 8


def build_sanitized(out: str) -> str:
    """The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
    (any report aborts), for the sanitizer test; load it by setting
    ORACLE_LIB=out (and preloading gcc's libasan) in a fresh process."""
    subprocess.check_call(
        ["gcc", "-O1", "-g", "-std=gnu11", "-Wall", "-ffp-contract=off", "-shared", "-fPIC",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
         "-o", out, _SRC, "-lm"])
    return out


def build(force: bool = False) -> str:
    """Compile the oracle with the host C compiler (no GPU code involved);
    ORACLE_LIB names another build to load instead (a sanitized one)."""
    if os.environ.get("ORACLE_LIB"):
        return os.environ["ORACLE_LIB"]
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
        os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "rapid_oracle.h"))
    ):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=gnu11", "-Wall", "-ffp-contract=off", "-shared", "-fPIC", "-o", tmp,
             _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


class OrcParams(C.Structure):
    _fields_ = [
        ("K", C.c_int32), ("gx", C.c_int32), ("gy", C.c_int32),
        ("n_levels", C.c_int32),
        ("factor", C.c_int32 * MAX_LEVELS),
        ("n_stages", C.c_int32 * MAX_LEVELS),
        ("stages", (C.c_int32 * MAX_STAGES) * MAX_LEVELS),
        ("gate_level", C.c_int32), ("frac_bits", C.c_int32),
        ("max_sweeps", C.c_int32), ("shuffle_seed", C.c_int32), ("gate_rule", C.c_int32),
        ("merge", C.c_int32), ("pad_", C.c_int32),
        ("min_size", C.c_int64), ("max_size", C.c_int64),
        ("w_col", C.c_int64), ("w_pos", C.c_int64), ("w_bnd", C.c_int64),
    ]


class OrcStageReport(C.Structure):
    _fields_ = [
        ("level", C.c_int32), ("block", C.c_int32), ("sweeps", C.c_int32),
        ("converged", C.c_int32), ("active", C.c_int64), ("proposals", C.c_int64),
        ("commits", C.c_int64), ("skip_min", C.c_int64), ("skip_topo", C.c_int64),
        ("merges", C.c_int64),
    ]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        L = _lib
        P = C.c_void_p
        L.orc_grid.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.orc_init_labels.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, P]
        L.orc_simple.argtypes = [C.c_int32]
        L.orc_segment.argtypes = [P, C.c_int32, C.c_int32, C.c_int64, C.POINTER(OrcParams), P,
                                  P, P, P, C.c_int32, C.c_int32]
        L.orc_propose_class.argtypes = [P, C.c_int32, C.c_int32, C.c_int64, C.POINTER(OrcParams), P,
                                        C.c_int32, C.c_int32, C.c_int32, P, P, P, C.c_int32]
        L.orc_block_energy.argtypes = [P, C.c_int32, C.c_int32, C.c_int64, C.POINTER(OrcParams), P,
                                       C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32]
        L.orc_block_energy.restype = C.c_int64
        L.orc_segment_ex.argtypes = [P, C.c_int32, C.c_int32, C.c_int64, C.POINTER(OrcParams), P,
                                     P, P, P, C.c_int32, C.c_int32, P, P]
        L.orc_segment_fifo.argtypes = [P, C.c_int32, C.c_int32, C.c_int64, C.POINTER(OrcParams), P, P, P,
                                       C.c_int32]
        L.orc_energy.argtypes = [P, C.c_int32, C.c_int32, C.c_int64, C.POINTER(OrcParams), P, C.c_int32]
        L.orc_energy.restype = C.c_int64
        L.orc_merge_cost.argtypes = [P, C.c_int32, C.c_int32, C.c_int64, C.POINTER(OrcParams), P,
                                     C.c_int32, C.c_int32, C.c_int32]
        L.orc_merge_cost.restype = C.c_int64
        L.orc_features.argtypes = [P, C.c_int32, C.c_int32, C.c_int64, P, C.c_int32, P, P,
                                   C.c_int32, C.c_int32, C.c_int32, P]
        L.orc_roi_features.argtypes = [P, C.c_int32, C.c_int32, C.c_int64, P, P, C.c_int32, C.c_int32,
                                       C.c_int32, P]
    return _lib


def make_params(d: dict, shuffle_seed: int = 0) -> OrcParams:
    p = OrcParams()
    p.K = int(d.get("K", 0))
    p.gx = int(d.get("gx", 0))
    p.gy = int(d.get("gy", 0))
    levels = d["levels"]
    p.n_levels = len(levels)
    for l, (f, st) in enumerate(levels):
        p.factor[l] = int(f)
        p.n_stages[l] = len(st)
        for s, b in enumerate(st):
            p.stages[l][s] = int(b)
    p.gate_level = int(d.get("gate_level", -1))
    p.frac_bits = int(d.get("frac_bits", 4))
    p.max_sweeps = int(d.get("max_sweeps", 64))
    p.shuffle_seed = int(shuffle_seed)
    p.gate_rule = GATE_RULES[d.get("gate_rule", "either")]
    p.merge = int(bool(d.get("merge", False)))
    p.min_size = int(d["min_size"])
    p.max_size = int(d["max_size"])
    p.w_col = int(d["w_col"])
    p.w_pos = int(d["w_pos"])
    p.w_bnd = int(d["w_bnd"])
    return p


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def grid(W: int, H: int, K: int):
    gx, gy = C.c_int32(), C.c_int32()
    rc = lib().orc_grid(W, H, K, C.byref(gx), C.byref(gy))
    if rc:
        raise ValueError("orc_grid rc=%d" % rc)
    return gx.value, gy.value


def init_labels(W: int, H: int, B0: int, gx: int, gy: int) -> np.ndarray:
    out = np.empty((H, W), np.int32)
    rc = lib().orc_init_labels(W, H, B0, gx, gy, _ptr(out))
    if rc:
        raise ValueError("orc_init_labels rc=%d" % rc)
    return out


def simple(mask: int) -> bool:
    return bool(lib().orc_simple(mask))


def n_superpixels(W: int, H: int, d: dict) -> int:
    if d.get("K", 0) > 0:
        gx, gy = grid(W, H, d["K"])
    else:
        gx, gy = d["gx"], d["gy"]
    return gx * gy


def segment(rgb: np.ndarray, d: dict, gate: np.ndarray | None = None,
            debug: bool = False, shuffle_seed: int = 0, track: bool = False):
    """Run the full schedule.  rgb: (H, W, 3) uint8.  Returns (labels (H, W)
    int32, stats (K', 6) int64, list of per-stage report dicts); with track,
    also involved (K',) uint8 (source or target of a proposal at a level >=
    gate_level) and moved (K',) int64 (pixels moved in or out)."""
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    H, W, _ = rgb.shape
    K = n_superpixels(W, H, d)
    labels = np.empty((H, W), np.int32)
    stats = np.empty((K, 6), np.int64)
    nst = sum(len(st) for _, st in d["levels"])
    reps = (OrcStageReport * max(nst, 1))()
    p = make_params(d, shuffle_seed)
    g = None
    if gate is not None:
        g = np.ascontiguousarray(gate, dtype=np.uint8)
        assert g.shape == (K,)
    inv = np.zeros(K, np.uint8) if track else None
    mov = np.zeros(K, np.int64) if track else None
    rc = lib().orc_segment_ex(_ptr(rgb), W, H, 3 * W, C.byref(p), _ptr(g), _ptr(labels),
                              _ptr(stats), reps, nst, int(debug), _ptr(inv), _ptr(mov))
    if rc < 0:
        raise RuntimeError("orc_segment failed rc=%d" % rc)
    out = (labels, stats, [reps[i].as_dict() for i in range(rc)])
    return out + (inv, mov) if track else out


def segment_fifo(rgb: np.ndarray, d: dict, debug: bool = False):
    """Sequential FIFO-queue schedule (see orc_segment_fifo): (labels,
    stats, moves)."""
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    H, W, _ = rgb.shape
    K = n_superpixels(W, H, d)
    labels = np.empty((H, W), np.int32)
    stats = np.empty((K, 6), np.int64)
    moves = C.c_int64(0)
    rc = lib().orc_segment_fifo(_ptr(rgb), W, H, 3 * W, C.byref(make_params(d)), _ptr(labels), _ptr(stats),
                                C.byref(moves), int(debug))
    if rc < 0:
        raise RuntimeError("orc_segment_fifo failed rc=%d" % rc)
    return labels, stats, int(moves.value)


def energy(rgb: np.ndarray, d: dict, labels: np.ndarray) -> int:
    """Eq. (1) at pixel level for a label map (see orc_energy)."""
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    H, W, _ = rgb.shape
    K = n_superpixels(W, H, d)
    return int(lib().orc_energy(_ptr(rgb), W, H, 3 * W, C.byref(make_params(d)), _ptr(labels), K))


def merge_cost(rgb: np.ndarray, d: dict, labels: np.ndarray, K: int, m: int, k: int) -> int:
    """Energy change of Eq. (1) when superpixel m is merged into k, for
    pixel labels labels (see orc_merge_cost)."""
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    H, W, _ = rgb.shape
    p = make_params(d)
    return int(lib().orc_merge_cost(_ptr(rgb), W, H, 3 * W, C.byref(p), _ptr(labels), K, m, k))


def features(rgb: np.ndarray, labels: np.ndarray, B: int, stats: np.ndarray,
             moved: np.ndarray | None, gx: int, gy: int, F: int = 4) -> np.ndarray:
    """Sixteen gate features per superpixel (see orc_features)."""
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    stats = np.ascontiguousarray(stats, dtype=np.int64)
    H, W, _ = rgb.shape
    K = gx * gy
    out = np.empty((K, 16), np.float32)
    mv = None if moved is None else np.ascontiguousarray(moved, dtype=np.int64)
    rc = lib().orc_features(_ptr(rgb), W, H, 3 * W, _ptr(labels), B, _ptr(stats), _ptr(mv),
                            gx, gy, F, _ptr(out))
    if rc < 0:
        raise RuntimeError("orc_features failed rc=%d" % rc)
    return out


def roi_features(rgb: np.ndarray, labels: np.ndarray, stats: np.ndarray, gx: int, gy: int,
                 F: int = 4) -> np.ndarray:
    """The paper's four ROI features per superpixel in 16-wide rows (see
    orc_roi_features)."""
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    stats = np.ascontiguousarray(stats, dtype=np.int64)
    H, W, _ = rgb.shape
    out = np.empty((gx * gy, 16), np.float32)
    rc = lib().orc_roi_features(_ptr(rgb), W, H, 3 * W, _ptr(labels), _ptr(stats), gx, gy, F, _ptr(out))
    if rc < 0:
        raise RuntimeError("orc_roi_features failed rc=%d" % rc)
    return out


def propose_class(rgb: np.ndarray, d: dict, labels: np.ndarray, K: int, B: int, cls: int,
                  gate: np.ndarray | None = None):
    """Proposals of one class for an arbitrary state (pixel labels); all
    eligible blocks active, statistics recounted.  Returns (N, 3) int32 of
    (block index, from, to) and (N,) int64 energy changes."""
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    H, W, _ = rgb.shape
    nbx, nby = -(-W // B), -(-H // B)
    cap = ((nbx + 2) // 3) * ((nby + 2) // 3)
    props = np.empty((cap, 3), np.int32)
    de = np.empty(cap, np.int64)
    g = None if gate is None else np.ascontiguousarray(gate, dtype=np.uint8)
    p = make_params(d)
    rc = lib().orc_propose_class(_ptr(rgb), W, H, 3 * W, C.byref(p), _ptr(labels), K, B, cls,
                                 _ptr(g), _ptr(props), _ptr(de), cap)
    if rc < 0:
        raise RuntimeError("orc_propose_class failed rc=%d" % rc)
    return props[:rc].copy(), de[:rc].copy()


def block_energy(rgb: np.ndarray, d: dict, labels: np.ndarray, K: int, B: int,
                 bx: int, by: int, k: int) -> int:
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    H, W, _ = rgb.shape
    p = make_params(d)
    return int(lib().orc_block_energy(_ptr(rgb), W, H, 3 * W, C.byref(p), _ptr(labels), K, B,
                                      bx, by, k))
