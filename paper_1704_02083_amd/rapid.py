"""Python binding of the C-ABI in ``include/rapid.h`` (``librapid.so``).

Argument marshalling only: every step of the segmentation runs in the HIP
kernels of the library.  PyTorch supplies device memory and the stream.
Importing this module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# RAPID_LIB selects another build of the same C-ABI (e.g. an instrumented one)
LIB_PATH = os.environ.get("RAPID_LIB") or os.path.join(_HERE, "librapid.so")

ABI_VERSION = 2
MAX_LEVELS = 4
MAX_STAGES = 8

if not os.path.exists(LIB_PATH):
    raise ImportError("librapid.so is not built (run __graft_entry__.build()): " + LIB_PATH)
_lib = C.CDLL(LIB_PATH)

STATUS = {0: "ok", -1: "invalid argument", -2: "out of memory", -3: "device error",
          -4: "state used out of order", -5: "gate model unusable"}


class RapidError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__("%s: %s (%d)" % (where, STATUS.get(code, "?"), code))
        self.code = code


CFG_TIMING = 1
CFG_AUTOTUNE = 2
CFG_TEST_ABORT = 4


class Config(C.Structure):
    _fields_ = [("abi_version", C.c_int32), ("device", C.c_int32), ("hip_stream", C.c_void_p),
                ("flags", C.c_int32), ("reserved", C.c_int32), ("autotune_cache", C.c_char_p)]


class Timings(C.Structure):
    _fields_ = [("block_sums_ms", C.c_float), ("refine_ms", C.c_float), ("threads", C.c_int32),
                ("stats_lds", C.c_int32), ("pyramid", C.c_int32), ("tuned", C.c_int32),
                ("workgroups", C.c_int32)]


class Params(C.Structure):
    _fields_ = [
        ("K", C.c_int32), ("gx", C.c_int32), ("gy", C.c_int32), ("n_levels", C.c_int32),
        ("factor", C.c_int32 * MAX_LEVELS), ("n_stages", C.c_int32 * MAX_LEVELS),
        ("stages", (C.c_int32 * MAX_STAGES) * MAX_LEVELS),
        ("gate_level", C.c_int32), ("frac_bits", C.c_int32), ("max_sweeps", C.c_int32),
        ("gate_rule", C.c_int32), ("merge", C.c_int32), ("gate_features", C.c_int32),
        ("min_size", C.c_int64), ("max_size", C.c_int64),
        ("w_col", C.c_int64), ("w_pos", C.c_int64), ("w_bnd", C.c_int64),
    ]


class Image(C.Structure):
    _fields_ = [("rgb_dev", C.c_void_p), ("W", C.c_int32), ("H", C.c_int32),
                ("row_stride_bytes", C.c_int64), ("labels_dev", C.c_void_p),
                ("label_stride", C.c_int64)]


class StageReport(C.Structure):
    _fields_ = [("level", C.c_int32), ("block", C.c_int32), ("sweeps", C.c_int32),
                ("converged", C.c_int32), ("active", C.c_int64), ("proposals", C.c_int64),
                ("commits", C.c_int64), ("skip_min", C.c_int64), ("skip_topo", C.c_int64),
                ("merges", C.c_int64)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class Report(C.Structure):
    _fields_ = [("n_stages", C.c_int32), ("K", C.c_int32),
                ("stage", StageReport * (MAX_LEVELS * MAX_STAGES))]

    def stages(self):
        return [self.stage[i].as_dict() for i in range(self.n_stages)]


class GateModel(C.Structure):
    _fields_ = [("w_bf16_dev", C.c_void_p), ("thresh", C.c_float)]


class TrainCfg(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("seed", C.c_uint64)]


class Slide(C.Structure):
    _fields_ = [("rgb_dev", C.c_void_p), ("W", C.c_int64), ("H", C.c_int64),
                ("row_stride_bytes", C.c_int64), ("labels_dev", C.c_void_p),
                ("label_stride", C.c_int64), ("tile", C.c_int32), ("halo", C.c_int32),
                ("cell", C.c_int32), ("reserved", C.c_int32)]


MLP_PARAMS = 5313
N_FEATURES = 16

_P = C.c_void_p
_lib.rapid_init.argtypes = [C.POINTER(Config), C.POINTER(_P)]
_lib.rapid_destroy.argtypes = [_P]
_lib.rapid_destroy.restype = None
_lib.rapid_segment.argtypes = [_P, C.POINTER(Image), C.POINTER(Params), _P, C.POINTER(Report)]
_lib.rapid_segment_batch.argtypes = [_P, C.POINTER(Image), C.c_int32, C.POINTER(Params),
                                     C.POINTER(Report)]
_lib.rapid_segment_noalloc.argtypes = [_P, C.POINTER(Image), C.POINTER(Params), _P, C.POINTER(Report)]
_lib.rapid_state_create.argtypes = [_P, C.POINTER(Image), C.POINTER(Params), C.POINTER(_P)]
_lib.rapid_refine_level.argtypes = [_P, _P, C.c_int32, _P, C.POINTER(Report)]
_lib.rapid_state_export.argtypes = [_P, _P, _P, _P]
_lib.rapid_state_destroy.argtypes = [_P]
_lib.rapid_state_destroy.restype = None
_lib.rapid_grid.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                            C.POINTER(C.c_int32)]
_lib.rapid_status_str.argtypes = [C.c_int]
_lib.rapid_status_str.restype = C.c_char_p
_lib.rapid_simple_lut.argtypes = [C.POINTER(C.c_uint32)]
_lib.rapid_check_params.argtypes = [C.c_int32, C.c_int32, C.POINTER(Params), C.POINTER(C.c_int32)]
_lib.rapid_last_timings.argtypes = [_P, C.POINTER(Timings)]
_lib.rapid_timing_history.argtypes = [_P, C.POINTER(C.c_float), C.c_int32, C.POINTER(C.c_int32)]
_lib.rapid_segment_gated.argtypes = [_P, C.POINTER(Image), C.c_int32, C.POINTER(Params),
                                     C.POINTER(GateModel), _P, _P, C.POINTER(Report)]
_lib.rapid_state_track.argtypes = [_P, _P, _P]
_lib.rapid_state_features.argtypes = [_P, _P, _P]
_lib.rapid_state_import.argtypes = [_P, _P, C.c_int32, _P, _P]
_lib.rapid_gate.argtypes = [_P, _P, C.POINTER(GateModel), _P, _P]
_lib.rapid_boundary_miss.argtypes = [_P, _P, _P, C.c_int32, C.c_int32, C.c_int64, C.c_int32, C.c_int32,
                                     _P, _P]
_lib.rapid_mlp_forward.argtypes = [_P, _P, C.c_int64, _P, C.c_float, _P, _P]
_lib.rapid_mlp_grad.argtypes = [_P, _P, _P, _P, C.c_int32, _P, _P, _P]
_lib.rapid_gate_train.argtypes = [_P, _P, _P, C.c_int64, C.POINTER(TrainCfg), _P, _P]
_lib.rapid_slide_tiles.argtypes = [C.POINTER(Slide), C.POINTER(C.c_int32)]
_lib.rapid_segment_slide.argtypes = [_P, C.POINTER(Slide), C.POINTER(Params), C.POINTER(GateModel),
                                     C.POINTER(Report)]
_lib.rapid_segment_slide_gated.argtypes = [_P, C.POINTER(Slide), C.POINTER(Params), C.POINTER(GateModel),
                                           _P, _P, C.POINTER(Report)]

EXPORTED = ["rapid_init", "rapid_destroy", "rapid_segment", "rapid_segment_batch",
            "rapid_state_create", "rapid_refine_level", "rapid_state_export",
            "rapid_state_destroy", "rapid_grid", "rapid_status_str", "rapid_simple_lut",
            "rapid_check_params", "rapid_last_timings", "rapid_segment_gated",
            "rapid_state_track", "rapid_state_features", "rapid_mlp_forward", "rapid_mlp_grad",
            "rapid_gate_train", "rapid_slide_tiles", "rapid_segment_slide", "rapid_boundary_miss",
            "rapid_state_import", "rapid_gate", "rapid_segment_slide_gated", "rapid_segment_noalloc",
            "rapid_timing_history"]


def _check(rc: int, where: str):
    if rc != 0:
        raise RapidError(rc, where)


GATE_RULES = {"either": 0, "both": 1, "differ": 2}   # RAPID_GATE_*
GATE_FEATURES = {"learned": 0, "roi": 1}              # RAPID_FEATURES_*


def make_params(d: dict) -> Params:
    p = Params()
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
    p.gate_rule = GATE_RULES[d.get("gate_rule", "either")]
    p.merge = int(bool(d.get("merge", False)))
    p.gate_features = GATE_FEATURES[d.get("gate_features", "learned")]
    p.min_size = int(d["min_size"])
    p.max_size = int(d["max_size"])
    p.w_col = int(d["w_col"])
    p.w_pos = int(d["w_pos"])
    p.w_bnd = int(d["w_bnd"])
    return p


# ----------------------------------------------------------- host helpers

def grid(W: int, H: int, K: int):
    gx, gy = C.c_int32(), C.c_int32()
    _check(_lib.rapid_grid(W, H, K, C.byref(gx), C.byref(gy)), "rapid_grid")
    return gx.value, gy.value


def simple_lut() -> list:
    out = (C.c_uint32 * 8)()
    _check(_lib.rapid_simple_lut(out), "rapid_simple_lut")
    return [int(v) for v in out]


def slide_tiles(W: int, H: int, tile: int, halo: int, cell: int) -> int:
    sl = Slide(None, W, H, 3 * W, None, W, tile, halo, cell, 0)
    n = C.c_int32()
    _check(_lib.rapid_slide_tiles(C.byref(sl), C.byref(n)), "rapid_slide_tiles")
    return n.value


def tile_layout(W: int, H: int, tile: int, halo: int, cell: int):
    """Tiles of a slide as dicts (core and extended rectangles, grid and the
    slide-cell offset of the grid), in the library's row-major order."""
    out = []
    for ty in range(-(-H // tile)):
        for tx in range(-(-W // tile)):
            cx0, cy0 = tx * tile, ty * tile
            cx1, cy1 = min(cx0 + tile, W), min(cy0 + tile, H)
            ex0, ey0 = max(0, cx0 - halo), max(0, cy0 - halo)
            ex1, ey1 = min(W, cx1 + halo), min(H, cy1 + halo)
            out.append({"core": (cx0, cy0, cx1, cy1), "ext": (ex0, ey0, ex1, ey1),
                        "gx": max(1, (ex1 - ex0) // cell), "gy": max(1, (ey1 - ey0) // cell),
                        "gid_x0": ex0 // cell, "gid_y0": ey0 // cell, "gid_w": -(-W // cell)})
    return out


def check_params(W: int, H: int, d: dict) -> int:
    """Validate params for a W x H image; returns the superpixel count."""
    k = C.c_int32()
    p = make_params(d)
    _check(_lib.rapid_check_params(W, H, C.byref(p), C.byref(k)), "rapid_check_params")
    return k.value


# -------------------------------------------------------------- device API

def _image(rgb, labels) -> Image:
    import torch
    assert rgb.is_cuda and rgb.dtype == torch.uint8 and rgb.dim() == 3 and rgb.shape[2] == 3
    assert rgb.stride(2) == 1 and rgb.stride(1) == 3, "rgb must be HWC with packed pixels"
    im = Image()
    im.rgb_dev = rgb.data_ptr()
    im.H, im.W = int(rgb.shape[0]), int(rgb.shape[1])
    im.row_stride_bytes = int(rgb.stride(0))
    if labels is not None:
        assert labels.is_cuda and labels.dtype == torch.int32 and labels.stride(1) == 1
        im.labels_dev = labels.data_ptr()
        im.label_stride = int(labels.stride(0))
    return im


class Context:
    """rapid_init / rapid_destroy around one device and stream."""

    def __init__(self, device: int = 0, stream=None, timing: bool = False, autotune: bool = False,
                 autotune_cache: str | None = None, test_abort: bool = False):
        import torch
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self._cache = autotune_cache.encode() if autotune_cache else None
        cfg = Config(ABI_VERSION, device, C.c_void_p(stream.cuda_stream),
                     (CFG_TIMING if timing else 0) | (CFG_AUTOTUNE if autotune else 0) |
                     (CFG_TEST_ABORT if test_abort else 0), 0, self._cache)
        h = _P()
        _check(_lib.rapid_init(C.byref(cfg), C.byref(h)), "rapid_init")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.rapid_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # rapid_segment
    def segment(self, rgb, params: dict, gate=None, labels=None, report: bool = True):
        import torch
        H, W = int(rgb.shape[0]), int(rgb.shape[1])
        if labels is None:
            labels = torch.empty((H, W), dtype=torch.int32, device=rgb.device)
        im = _image(rgb, labels)
        p = make_params(params)
        rep = Report() if report else None
        g = None if gate is None else C.c_void_p(gate.data_ptr())
        _check(_lib.rapid_segment(self._h, C.byref(im), C.byref(p), g,
                                  C.byref(rep) if rep is not None else None), "rapid_segment")
        return labels, (rep.stages() if rep is not None else None)

    # rapid_segment_noalloc: as segment, with the library's fixed scratch
    # (the caller passes the output labels to allocate nothing at all)
    def segment_noalloc(self, rgb, params: dict, gate=None, labels=None, report: bool = True):
        import torch
        H, W = int(rgb.shape[0]), int(rgb.shape[1])
        if labels is None:
            labels = torch.empty((H, W), dtype=torch.int32, device=rgb.device)
        im = _image(rgb, labels)
        p = make_params(params)
        rep = Report() if report else None
        g = None if gate is None else C.c_void_p(gate.data_ptr())
        _check(_lib.rapid_segment_noalloc(self._h, C.byref(im), C.byref(p), g,
                                          C.byref(rep) if rep is not None else None), "rapid_segment_noalloc")
        return labels, (rep.stages() if rep is not None else None)

    # rapid_segment_batch
    def segment_batch(self, rgbs, params: dict, labels=None, report: bool = True):
        import torch
        n = len(rgbs)
        if labels is None:
            labels = [torch.empty((int(r.shape[0]), int(r.shape[1])), dtype=torch.int32,
                                  device=r.device) for r in rgbs]
        ims = (Image * n)(*[_image(r, l) for r, l in zip(rgbs, labels)])
        p = make_params(params)
        reps = (Report * n)() if report else None
        _check(_lib.rapid_segment_batch(self._h, ims, n, C.byref(p), reps), "rapid_segment_batch")
        return labels, ([r.stages() for r in reps] if reps is not None else None)

    # rapid_segment_gated
    def segment_gated(self, rgbs, params: dict, w_bf16, thresh: float = 0.0, labels=None,
                      features: bool = False, report: bool = True):
        """Returns (labels list, reports, features (sum K, 16) or None, gate bits)."""
        import torch
        n = len(rgbs)
        if labels is None:
            labels = [torch.empty((int(r.shape[0]), int(r.shape[1])), dtype=torch.int32,
                                  device=r.device) for r in rgbs]
        ims = (Image * n)(*[_image(r, l) for r, l in zip(rgbs, labels)])
        p = make_params(params)
        Ktot = sum(check_params(int(r.shape[1]), int(r.shape[0]), params) for r in rgbs)
        X = torch.empty((Ktot, N_FEATURES), dtype=torch.float32, device=rgbs[0].device) if features else None
        g = torch.empty(Ktot, dtype=torch.uint8, device=rgbs[0].device)
        model = GateModel(w_bf16.data_ptr(), thresh)
        reps = (Report * n)() if report else None
        rc = _lib.rapid_segment_gated(self._h, ims, n, C.byref(p), C.byref(model),
                                      C.c_void_p(X.data_ptr()) if X is not None else None,
                                      C.c_void_p(g.data_ptr()), reps)
        _check(rc, "rapid_segment_gated")
        return labels, ([r.stages() for r in reps] if reps is not None else None), X, g

    # rapid_segment_slide
    def segment_slide(self, rgb, params: dict, tile: int = 2048, halo: int = 64, cell: int = 32,
                      labels=None, w_bf16=None, thresh: float = 0.0, report: bool = False,
                      features: bool = False):
        """rapid_segment_slide (plain, or gated with w_bf16); with features
        (gated only) rapid_segment_slide_gated, and the result gains the
        feature rows (sum of tile K, 16) and gate bytes of every tile's
        superpixels in tile order."""
        import torch
        H, W = int(rgb.shape[0]), int(rgb.shape[1])
        assert rgb.is_cuda and rgb.dtype == torch.uint8 and rgb.stride(1) == 3 and rgb.stride(2) == 1
        if labels is None:
            labels = torch.empty((H, W), dtype=torch.int32, device=rgb.device)
        sl = Slide(rgb.data_ptr(), W, H, int(rgb.stride(0)), labels.data_ptr(), int(labels.stride(0)),
                   tile, halo, cell, 0)
        nt = slide_tiles(W, H, tile, halo, cell)
        p = make_params(dict(params, K=0, gx=1, gy=1))
        model = GateModel(w_bf16.data_ptr(), thresh) if w_bf16 is not None else None
        reps = (Report * nt)() if report else None
        if features:
            assert model is not None, "features come from the gated route"
            Kt = sum(t["gx"] * t["gy"] for t in tile_layout(W, H, tile, halo, cell))
            X = torch.empty((Kt, N_FEATURES), dtype=torch.float32, device=rgb.device)
            g = torch.empty(Kt, dtype=torch.uint8, device=rgb.device)
            _check(_lib.rapid_segment_slide_gated(self._h, C.byref(sl), C.byref(p), C.byref(model),
                                                  C.c_void_p(X.data_ptr()), C.c_void_p(g.data_ptr()), reps),
                   "rapid_segment_slide_gated")
            return labels, ([r.stages() for r in reps] if reps is not None else None), X, g
        _check(_lib.rapid_segment_slide(self._h, C.byref(sl), C.byref(p),
                                        C.byref(model) if model is not None else None, reps),
               "rapid_segment_slide")
        return labels, ([r.stages() for r in reps] if reps is not None else None)

    def boundary_miss(self, ref, test, radius: int = 2, K: int = 0, counts: bool = True):
        """Boundary-recall misses of test against ref (two (H, W) int32
        device maps with the same strides).  Returns (per-label counts (K,)
        int32 or None, ref boundary pixels, missed pixels)."""
        import torch
        assert ref.shape == test.shape and ref.stride() == test.stride() and ref.stride(1) == 1
        H, W = int(ref.shape[0]), int(ref.shape[1])
        miss = torch.zeros(K, dtype=torch.int32, device=ref.device) if counts else None
        tot = torch.zeros(2, dtype=torch.int64, device=ref.device)
        _check(_lib.rapid_boundary_miss(self._h, C.c_void_p(ref.data_ptr()), C.c_void_p(test.data_ptr()), W, H,
                                        int(ref.stride(0)), radius, K,
                                        C.c_void_p(miss.data_ptr()) if miss is not None else None,
                                        C.c_void_p(tot.data_ptr())), "rapid_boundary_miss")
        t = tot.cpu()
        return miss, int(t[0]), int(t[1])

    def mlp_forward(self, X, w_bf16, thresh: float = 0.0):
        import torch
        n = int(X.shape[0])
        logits = torch.empty(n, dtype=torch.float32, device=X.device)
        gate = torch.empty(n, dtype=torch.uint8, device=X.device)
        _check(_lib.rapid_mlp_forward(self._h, C.c_void_p(X.data_ptr()), n, C.c_void_p(w_bf16.data_ptr()),
                                      thresh, C.c_void_p(logits.data_ptr()), C.c_void_p(gate.data_ptr())),
               "rapid_mlp_forward")
        return logits, gate

    def mlp_grad(self, X, t, idx, w_bf16):
        import torch
        grads = torch.empty(MLP_PARAMS, dtype=torch.float32, device=X.device)
        logits = torch.empty(int(idx.shape[0]), dtype=torch.float32, device=X.device)
        _check(_lib.rapid_mlp_grad(self._h, C.c_void_p(X.data_ptr()), C.c_void_p(t.data_ptr()),
                                   C.c_void_p(idx.data_ptr()), int(idx.shape[0]),
                                   C.c_void_p(w_bf16.data_ptr()), C.c_void_p(grads.data_ptr()),
                                   C.c_void_p(logits.data_ptr())), "rapid_mlp_grad")
        return grads, logits

    def gate_train(self, X, t, master, epochs: int = 20, batch: int = 4096, lr: float = 1e-3,
                   beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, seed: int = 0):
        """Trains in place: master (5313 float32, device) in/out; returns the
        bf16 weights (5313 uint16 as int16 tensor)."""
        import torch
        w = torch.empty(MLP_PARAMS, dtype=torch.int16, device=X.device)
        cfg = TrainCfg(epochs, batch, lr, beta1, beta2, eps, seed)
        _check(_lib.rapid_gate_train(self._h, C.c_void_p(X.data_ptr()), C.c_void_p(t.data_ptr()),
                                     int(X.shape[0]), C.byref(cfg), C.c_void_p(master.data_ptr()),
                                     C.c_void_p(w.data_ptr())), "rapid_gate_train")
        return w

    def last_timings(self) -> dict:
        t = Timings()
        _check(_lib.rapid_last_timings(self._h, C.byref(t)), "rapid_last_timings")
        return {"block_sums_ms": float(t.block_sums_ms), "refine_ms": float(t.refine_ms),
                "threads": int(t.threads), "stats_lds": int(t.stats_lds), "pyramid": int(t.pyramid),
                "tuned": int(t.tuned), "workgroups": int(t.workgroups)}

    def timing_history(self, n: int) -> list:
        """rapid_timing_history: refinement kernel durations (ms) of the last
        n timed calls (at most 128), oldest first."""
        buf = (C.c_float * max(n, 1))()
        got = C.c_int32()
        _check(_lib.rapid_timing_history(self._h, buf, n, C.byref(got)), "rapid_timing_history")
        return [float(buf[i]) for i in range(got.value)]

    def state(self, rgb, params: dict) -> "State":
        return State(self, rgb, params)


class State:
    """rapid_state_create / rapid_refine_level / rapid_gate / rapid_state_export /
    rapid_state_import."""

    def __init__(self, ctx: Context, rgb, params: dict):
        self.ctx = ctx
        self.rgb = rgb
        im = _image(rgb, None)
        p = make_params(params)
        h = _P()
        _check(_lib.rapid_state_create(ctx._h, C.byref(im), C.byref(p), C.byref(h)),
               "rapid_state_create")
        self._h = h
        self.K = check_params(im.W, im.H, params)

    def refine_level(self, level: int, gate=None, report: bool = True):
        rep = Report() if report else None
        g = None if gate is None else C.c_void_p(gate.data_ptr())
        _check(_lib.rapid_refine_level(self.ctx._h, self._h, level, g,
                                       C.byref(rep) if rep is not None else None),
               "rapid_refine_level")
        return rep.stages() if rep is not None else None

    def track(self, involved=None, moved=None):
        _check(_lib.rapid_state_track(self._h,
                                      C.c_void_p(involved.data_ptr()) if involved is not None else None,
                                      C.c_void_p(moved.data_ptr()) if moved is not None else None),
               "rapid_state_track")

    def features(self):
        import torch
        X = torch.empty((self.K, N_FEATURES), dtype=torch.float32, device=self.rgb.device)
        _check(_lib.rapid_state_features(self.ctx._h, self._h, C.c_void_p(X.data_ptr())),
               "rapid_state_features")
        return X

    def gate(self, w_bf16, thresh: float = 0.0, features: bool = False, out=None):
        """rapid_gate: (gate bytes (K,), features (K, 16) or None); out: an
        optional (K,) uint8 tensor for the gate bytes."""
        import torch
        g = torch.empty(self.K, dtype=torch.uint8, device=self.rgb.device) if out is None else out
        assert g.is_cuda and g.dtype == torch.uint8 and g.numel() == self.K and g.is_contiguous()
        X = torch.empty((self.K, N_FEATURES), dtype=torch.float32, device=self.rgb.device) if features else None
        model = GateModel(w_bf16.data_ptr(), thresh)
        _check(_lib.rapid_gate(self.ctx._h, self._h, C.byref(model),
                               C.c_void_p(X.data_ptr()) if X is not None else None, C.c_void_p(g.data_ptr())),
               "rapid_gate")
        return g, X

    def import_(self, next_level: int, labels, stats=None):
        """rapid_state_import: labels (H, W) int32 and stats (K, 6) int64 or
        None, both contiguous on the state's device."""
        import torch
        H, W = int(self.rgb.shape[0]), int(self.rgb.shape[1])
        assert labels.is_cuda and labels.dtype == torch.int32 and tuple(labels.shape) == (H, W)
        assert labels.is_contiguous()
        if stats is not None:
            assert stats.is_cuda and stats.dtype == torch.int64 and tuple(stats.shape) == (self.K, 6)
            assert stats.is_contiguous()
        _check(_lib.rapid_state_import(self.ctx._h, self._h, next_level, C.c_void_p(labels.data_ptr()),
                                       C.c_void_p(stats.data_ptr()) if stats is not None else None),
               "rapid_state_import")

    def export(self):
        import torch
        H, W = int(self.rgb.shape[0]), int(self.rgb.shape[1])
        labels = torch.empty((H, W), dtype=torch.int32, device=self.rgb.device)
        stats = torch.empty((self.K, 6), dtype=torch.int64, device=self.rgb.device)
        _check(_lib.rapid_state_export(self.ctx._h, self._h, C.c_void_p(labels.data_ptr()),
                                       C.c_void_p(stats.data_ptr())), "rapid_state_export")
        return labels, stats

    def close(self):
        if getattr(self, "_h", None):
            _lib.rapid_state_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
