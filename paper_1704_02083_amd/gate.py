"""Training data, training and calibration of the prediction gate.

Every step runs on the GPU through the C-ABI (``rapid.py``): plain
refinements of training tiles produce the features (at the start of the
gate level) and the targets, ``rapid_gate_train`` fits the network, and
``rapid_segment_gated`` applies it.

Target (this project's reading of "which superpixels need refinement at
finer levels"): superpixel k is positive when the plain run moves at least
a fraction ``tau`` of its pixels into or out of it after the gate point.
"""
from __future__ import annotations

import numpy as np

from . import metrics, rapid


def tile_samples(ctx, rgb, p: dict, tau: float):
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
    _, stats = st.export()
    moved_gate = moved.clone()
    for l in range(gl, len(p["levels"])):
        st.refine_level(l, report=False)
    lab, _ = st.export()
    st.close()
    after = (moved - moved_gate).to(torch.float64)
    n = stats[:, 0].to(torch.float64)
    t = (after >= tau * n).to(torch.uint8)
    return X, t, lab


def training_set(ctx, rgbs, p: dict, tau: float):
    import torch
    Xs, ts = [], []
    for r in rgbs:
        X, t, _ = tile_samples(ctx, r, p, tau)
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


def evaluate(ctx, rgbs, p: dict, w, thresh: float, plain_labels=None, timing: bool = True):
    """Gated vs plain on the same images: agreement metrics and the share
    of superpixels the gate marks."""
    import torch
    if plain_labels is None:
        plain_labels, _ = ctx.segment_batch(rgbs, p, report=False)
    labs, _, _, g = ctx.segment_gated(rgbs, p, w, thresh, report=False)
    torch.cuda.synchronize()
    m = {"br": [], "ue": [], "disagreement": []}
    for a, b in zip(plain_labels, labs):
        r = metrics.agreement(a.cpu().numpy(), b.cpu().numpy())
        for k in m:
            m[k].append(r[k])
    out = {k: float(np.mean(v)) for k, v in m.items()}
    out["br_min"] = float(np.min(m["br"]))
    out["marked"] = float(g.to(torch.float32).mean().item())
    return out


def calibrate(ctx, rgbs, p: dict, w, target_br: float = 0.99, candidates=None):
    """Largest logit threshold whose mean boundary recall against the plain
    result is at least target_br on the given (held-out) images."""
    import torch
    plain, _ = ctx.segment_batch(rgbs, p, report=False)
    torch.cuda.synchronize()
    if candidates is None:
        candidates = [4.0, 3.0, 2.0, 1.5, 1.0, 0.5, 0.0, -0.5, -1.0, -2.0, -3.0, -4.0, -6.0, -8.0]
    best = None
    for th in candidates:
        r = evaluate(ctx, rgbs, p, w, th, plain_labels=plain)
        if r["br"] >= target_br:
            best = (th, r)
            break
    return best
