"""Reference of the gate network (Eq. (6): y = 1 when h(x) >= 0).

TEST INFRASTRUCTURE ONLY (the product path never imports it).

h is a multilayer perceptron 16 -> 64 -> 64 -> 1 with ReLU and a logistic
output, trained with binary cross-entropy and Adam (Kingma & Ba, 2015).
Accumulation is fp64.  With ``bf16=True`` the operands are rounded to
bfloat16 (round to nearest even) exactly where the GPU rounds them: the
inputs, every weight and bias, the hidden activations fed to the next layer
and the back-propagated hidden gradients fed to the weight-gradient and
input-gradient products.  With ``bf16=False`` it is plain fp64 math, which
the central-difference test pins.

Parameter vector (5313 values): W1 (64 x 16, row = output), b1 (64),
W2 (64 x 64), b2 (64), w3 (64), b3 (1).
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 16, 64
SIZES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
         ("w3", (N_H,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)   # 5313


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def pack(parts: dict) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], np.float64).ravel() for name, _ in SIZES])


def bf16_round(x) -> np.ndarray:
    """fp32 -> bfloat16 -> fp32, round to nearest even (no NaN inputs)."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def to_bf16_bits(x) -> np.ndarray:
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def from_bf16_bits(b) -> np.ndarray:
    return (np.asarray(b, np.uint32) << 16).view(np.float32).astype(np.float64)


def _r(x, bf16):
    return bf16_round(x) if bf16 else np.asarray(x, np.float64)


def forward(theta: np.ndarray, X: np.ndarray, bf16: bool = True):
    """Returns the logits z (N,) and the cache for backward."""
    P = {k: _r(v, bf16) for k, v in unpack(theta).items()}
    x = _r(X, bf16)
    a1 = x @ P["W1"].T + P["b1"]
    h1 = _r(np.maximum(a1, 0.0), bf16)
    a2 = h1 @ P["W2"].T + P["b2"]
    h2 = _r(np.maximum(a2, 0.0), bf16)
    z = h2 @ P["w3"] + P["b3"][0]
    return z, (P, x, a1, h1, a2, h2)


def loss(theta, X, t, bf16=True) -> float:
    z, _ = forward(theta, X, bf16)
    t = np.asarray(t, np.float64)
    return float(np.mean(np.maximum(z, 0) - z * t + np.log1p(np.exp(-np.abs(z)))))


def grad(theta: np.ndarray, X: np.ndarray, t: np.ndarray, bf16: bool = True):
    """Gradient of the mean binary cross-entropy with logits."""
    z, (P, x, a1, h1, a2, h2) = forward(theta, X, bf16)
    n = X.shape[0]
    t = np.asarray(t, np.float64)
    dz = (1.0 / (1.0 + np.exp(-z)) - t) / n
    g = {}
    g["w3"] = h2.T @ dz
    g["b3"] = np.array([dz.sum()])
    dh2 = _r(np.outer(dz, P["w3"]) * (a2 > 0), bf16)
    g["W2"] = dh2.T @ h1
    g["b2"] = dh2.sum(0)
    dh1 = _r((dh2 @ P["W2"]) * (a1 > 0), bf16)
    g["W1"] = dh1.T @ x
    g["b1"] = dh1.sum(0)
    return pack(g), z


def adam_step(theta, m, v, g, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def he_init(seed: int) -> np.ndarray:
    """He-normal weights from a seed, zero biases."""
    rng = np.random.default_rng(seed)
    parts = {"W1": rng.normal(0, np.sqrt(2.0 / N_IN), (N_H, N_IN)),
             "b1": np.zeros(N_H),
             "W2": rng.normal(0, np.sqrt(2.0 / N_H), (N_H, N_H)),
             "b2": np.zeros(N_H),
             "w3": rng.normal(0, np.sqrt(1.0 / N_H), N_H),
             "b3": np.zeros(1)}
    return pack(parts)
