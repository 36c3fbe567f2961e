"""Training data, training and calibration of the prediction gate.

Every step runs on the GPU through the C-ABI (``rapid.py``): plain
refinements of training tiles produce the features at the gate point and the
targets, ``rapid_gate_train`` fits the network, and ``rapid_segment_gated``
applies it.

Target (this project's reading of "which superpixels need refinement at
finer levels"): superpixel k is positive when, in the plain run, at least
``min_miss`` boundary pixels charged to k (``rapid_boundary_miss``) end up
more than ``radius`` pixels away from every boundary pixel at the gate
point: freezing k there would cost boundary recall.
"""
from __future__ import annotations

import numpy as np

from . import rapid


def tile_samples(ctx, rgb, p: dict, radius: int = 2, min_miss: int = 1):
    """Plain run of one image through the level-by-level API.  Returns the
    gate features (K, 16), targets (K,) uint8 and the plain labels."""
    import torch
    st = ctx.state(rgb, p)
    K = st.K
    moved = torch.zeros(K, dtype=torch.int64, device=rgb.device)
    st.track(None, moved)
    gl = p["gate_level"]
    for l in range(gl):
        st.refine_level(l, report=False)
    X = st.features()
    lab_gate, _ = st.export()
    for l in range(gl, len(p["levels"])):
        st.refine_level(l, report=False)
    lab, _ = st.export()
    st.close()
    miss, _, _ = ctx.boundary_miss(lab, lab_gate, radius=radius, K=K)
    return X, (miss >= min_miss).to(torch.uint8), lab


def training_set(ctx, rgbs, p: dict, radius: int = 2, min_miss: int = 1):
    import torch
    Xs, ts = [], []
    for r in rgbs:
        X, t, _ = tile_samples(ctx, r, p, radius, min_miss)
        Xs.append(X)
        ts.append(t)
    return torch.cat(Xs), torch.cat(ts)


def init_master(seed: int):
    """He-normal weights (fp32) from a seed, zero biases, as a host array."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0, np.sqrt(2.0 / 16), (64, 16))
    W2 = rng.normal(0, np.sqrt(2.0 / 64), (64, 64))
    w3 = rng.normal(0, np.sqrt(1.0 / 64), 64)
    return np.concatenate([W1.ravel(), np.zeros(64), W2.ravel(), np.zeros(64), w3, [0.0]]).astype(np.float32)


def train(ctx, X, t, epochs: int = 20, batch: int = 4096, lr: float = 1e-3, seed: int = 0):
    import torch
    master = torch.from_numpy(init_master(seed)).to(X.device)
    batch = min(batch, 2 * (int(X.shape[0]) // 2))
    w = ctx.gate_train(X, t, master, epochs=epochs, batch=batch, lr=lr, seed=seed)
    return master, w


def save_model(path: str, master, w_bf16, thresh: float = 0.0, gate_level: int = 3, rule: str = "both"):
    """Write a trained gate to an .npz file (no pickled objects): the fp32
    master weights, their bf16 bit patterns, the threshold and the schedule
    point it was trained for."""
    np.savez(path, master=np.asarray(master.cpu().numpy() if hasattr(master, "cpu") else master,
                                     dtype=np.float32),
             w_bf16=np.asarray(w_bf16.cpu().numpy() if hasattr(w_bf16, "cpu") else w_bf16).view(np.int16),
             thresh=np.float64(thresh), gate_level=np.int32(gate_level), rule=np.array(rule))


def load_model(path: str, device="cuda"):
    """Read a gate written by save_model: (master fp32, w_bf16 int16 bit
    patterns as torch tensors on device, dict of threshold, gate level and
    rule).  The bf16 patterns must round the master weights to nearest even."""
    import torch
    with np.load(path, allow_pickle=False) as z:
        master, wb = z["master"], z["w_bf16"]
        meta = {"thresh": float(z["thresh"]), "gate_level": int(z["gate_level"]), "rule": str(z["rule"])}
    if master.shape != (5313,) or wb.shape != (5313,):
        raise ValueError("not a gate model: %s" % path)
    return torch.from_numpy(master).to(device), torch.from_numpy(wb).to(device), meta


def boundary_recall(ctx, ref, test, radius: int = 2) -> float:
    """Boundary recall of test against ref, on the GPU (any map size)."""
    _, nb, nm = ctx.boundary_miss(ref, test, radius=radius, counts=False)
    return 1.0 - nm / nb if nb else 1.0


def evaluate(ctx, rgbs, p: dict, w, thresh: float, plain_labels=None):
    """Gated vs plain on the same images: mean boundary recall, its minimum,
    the share of differing labels and the share of superpixels marked."""
    import torch
    if plain_labels is None:
        plain_labels, _ = ctx.segment_batch(rgbs, p, report=False)
    labs, _, _, g = ctx.segment_gated(rgbs, p, w, thresh, report=False)
    brs = [boundary_recall(ctx, a, b) for a, b in zip(plain_labels, labs)]
    dis = [float((a != b).float().mean().item()) for a, b in zip(plain_labels, labs)]
    return {"br": float(np.mean(brs)), "br_min": float(np.min(brs)), "disagreement": float(np.mean(dis)),
            "marked": float(g.to(torch.float32).mean().item())}


def calibrate(ctx, rgbs, p: dict, w, target_br: float = 0.99, candidates=None):
    """Largest logit threshold (fewest superpixels marked) whose mean
    boundary recall against the plain result is at least target_br on the
    given (held-out) images.  Returns (threshold, evaluation) or None."""
    plain, _ = ctx.segment_batch(rgbs, p, report=False)
    if candidates is None:
        candidates = [4.0, 3.0, 2.0, 1.5, 1.0, 0.5, 0.0, -0.5, -1.0, -1.5, -2.0, -3.0, -4.0, -6.0]
    for th in candidates:
        r = evaluate(ctx, rgbs, p, w, th, plain_labels=plain)
        if r["br"] >= target_br:
            return th, r
    return None


# ----------------------------------------------------- region of interest
#
# The paper's own prediction step: a classifier labels every superpixel ROI
# or not at the gate point, and past it only pairs of superpixels of
# different predicted classes refine (Eq. (7), rule "differ").  Here the
# classifier is the same network trained on "most of the superpixel's pixels
# lie in the region of interest" (on the synthetic H&E images: tissue, as
# opposed to background).

def roi_samples(ctx, rgb, roi, p: dict):
    """Plain run to the gate point: features (K, 16) and ROI targets (K,)
    uint8 (at least half of the superpixel's pixels in roi)."""
    import torch
    st = ctx.state(rgb, p)
    K = st.K
    moved = torch.zeros(K, dtype=torch.int64, device=rgb.device)
    st.track(None, moved)
    for l in range(p["gate_level"]):
        st.refine_level(l, report=False)
    X = st.features()
    lab, _ = st.export()
    st.close()
    lab = lab.reshape(-1).long()
    n = torch.bincount(lab, minlength=K)
    inside = torch.bincount(lab[roi.reshape(-1)], minlength=K)
    return X, (2 * inside >= n).to(torch.uint8)


def roi_mask(labels, gate):
    """Pixel ROI mask of a segmentation: the predicted class of each pixel's
    superpixel."""
    return gate[labels.long()].bool()


def roi_scores(pred, truth) -> dict:
    """Pixel precision, recall and F1 of a predicted ROI mask (Sec. 4's ROI
    detection measures)."""
    tp = int((pred & truth).sum().item())
    fp = int((pred & ~truth).sum().item())
    fn = int((~pred & truth).sum().item())
    prec = tp / (tp + fp) if tp + fp else 1.0
    rec = tp / (tp + fn) if tp + fn else 1.0
    f1 = 2 * prec * rec / (prec + rec) if prec + rec else 0.0
    return {"precision": prec, "recall": rec, "f1": f1}
