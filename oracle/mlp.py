"""CPU oracle of the change-predictor network -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this module.  It is the plain fp64 reference for the GPU's forward, backward
and Adam kernels and shares no code with them.

The network is a project addition (not in the paper): a multilayer perceptron
12 -> 64 -> 64 -> 1 with ReLU hidden layers and a sigmoid output that, from
per-vertex features, predicts whether a flagged vertex will change label when
processed.  Parameters are stored in bfloat16 (with fp32 master copies for the
optimiser); arithmetic here is fp64 on the bf16-rounded values.

  bf16_round(x)        round-to-nearest-even to bfloat16 (the top 16 bits of
                       an IEEE-754 binary32), returned as float32
  forward(p, X)        logits; also the hidden activations
  bce_loss(z, y, pw)   mean binary cross-entropy with logits, positive weight pw
  backward(p, X, y, pw) gradients of bce_loss w.r.t. every parameter
  adam_step(...)       one Adam update (Kingma & Ba 2015) with bias correction
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 12, 64
PARAM_SHAPES = {"W1": (N_IN, N_H), "b1": (N_H,), "W2": (N_H, N_H), "b2": (N_H,),
                "W3": (N_H, 1), "b3": (1,)}
PARAM_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def bf16_round(x) -> np.ndarray:
    """Round float32 values to the nearest bfloat16, ties to even; NaN stays
    NaN (quiet), infinities stay infinite.  Returned as float32."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    nan = np.isnan(a)
    r = np.where(nan, (u.astype(np.uint32) | 0x00400000) & 0xFFFF0000, r).astype(np.uint32)
    return r.view(np.float32).reshape(a.shape)


def init_params(seed: int) -> dict:
    """He-style uniform initialisation (fp32 master values)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in PARAM_SHAPES.items():
        if name.startswith("W"):
            lim = np.sqrt(6.0 / shp[0])
            p[name] = rng.uniform(-lim, lim, size=shp).astype(np.float32)
        else:
            p[name] = np.zeros(shp, dtype=np.float32)
    return p


def _w(a, exact):
    return np.asarray(a, dtype=np.float64) if exact else bf16_round(a).astype(np.float64)


def forward(p: dict, X: np.ndarray, bf16_h1: bool = False, exact: bool = False):
    """Logits z (shape [B]) and hidden activations (h1, h2), fp64.  Weights and
    inputs are taken at bf16 precision (exact=True: at their full value).  With
    bf16_h1 the first hidden layer's output, an operand of the second matrix
    product, is rounded to bf16 (through fp32) as in bf16 inference; the
    second hidden layer feeds only the final fp32 dot product and is never
    rounded.  Biases stay fp32."""
    W1, b1 = _w(p["W1"], exact), np.asarray(p["b1"], dtype=np.float64)
    W2, b2 = _w(p["W2"], exact), np.asarray(p["b2"], dtype=np.float64)
    W3, b3 = _w(p["W3"], exact), np.asarray(p["b3"], dtype=np.float64)
    x = _w(X, exact)
    a1 = x @ W1 + b1
    h1 = np.maximum(a1, 0.0)
    if bf16_h1:
        h1 = bf16_round(h1.astype(np.float32)).astype(np.float64)
    a2 = h1 @ W2 + b2
    h2 = np.maximum(a2, 0.0)
    z = (h2 @ W3 + b3)[:, 0]
    return z, (x, a1, h1, a2, h2)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def bce_loss(z: np.ndarray, y: np.ndarray, pos_weight: float = 1.0) -> float:
    """mean over samples of  -[pw * y * log s(z) + (1 - y) * log(1 - s(z))]."""
    z = np.asarray(z, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    log_s = -np.logaddexp(0.0, -z)      # log sigmoid(z)
    log_1ms = -np.logaddexp(0.0, z)     # log (1 - sigmoid(z))
    return float(np.mean(-(pos_weight * y * log_s + (1.0 - y) * log_1ms)))


def backward(p: dict, X: np.ndarray, y: np.ndarray, pos_weight: float = 1.0,
             bf16_h1: bool = False, exact: bool = False) -> dict:
    """Gradients of bce_loss(forward(p, X)) w.r.t. the parameters (chain rule
    through the layers; the bf16 rounding is treated as identity)."""
    z, (x, a1, h1, a2, h2) = forward(p, X, bf16_h1, exact)
    y = np.asarray(y, dtype=np.float64)
    B = z.shape[0]
    s = sigmoid(z)
    # d/dz of -[pw y log s + (1-y) log(1-s)] = pw y (s - 1) + (1 - y) s
    dz = (pos_weight * y * (s - 1.0) + (1.0 - y) * s) / B
    W2 = _w(p["W2"], exact)
    W3 = _w(p["W3"], exact)
    g = {}
    g["W3"] = h2.T @ dz[:, None]
    g["b3"] = np.array([dz.sum()])
    dh2 = dz[:, None] @ W3.T
    da2 = dh2 * (a2 > 0.0)
    g["W2"] = h1.T @ da2
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ W2.T
    da1 = dh1 * (a1 > 0.0)
    g["W1"] = x.T @ da1
    g["b1"] = da1.sum(axis=0)
    return g


def adam_step(p: dict, g: dict, m: dict, v: dict, t: int, lr: float = 1e-3,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
    """In place: m <- b1 m + (1-b1) g; v <- b2 v + (1-b2) g^2;
    p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
    t counts steps from 1.  Done in fp64, stored back as fp32."""
    for k in PARAM_ORDER:
        gk = np.asarray(g[k], dtype=np.float64)
        m[k] = (beta1 * m[k].astype(np.float64) + (1.0 - beta1) * gk).astype(np.float32)
        v[k] = (beta2 * v[k].astype(np.float64) + (1.0 - beta2) * gk * gk).astype(np.float32)
        mh = m[k].astype(np.float64) / (1.0 - beta1 ** t)
        vh = v[k].astype(np.float64) / (1.0 - beta2 ** t)
        p[k] = (p[k].astype(np.float64) - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32)


def flatten(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[k], dtype=np.float32).ravel() for k in PARAM_ORDER])


def unflatten(flat: np.ndarray) -> dict:
    out, o = {}, 0
    for k in PARAM_ORDER:
        n = int(np.prod(PARAM_SHAPES[k]))
        out[k] = np.asarray(flat[o:o + n], dtype=np.float32).reshape(PARAM_SHAPES[k])
        o += n
    return out


N_PARAMS = sum(int(np.prod(s)) for s in PARAM_SHAPES.values())  # 5,057
