"""FP64 reference of the scheduling cost model (test infrastructure only).

A 4 -> 64 -> 64 -> 1 ReLU MLP on standardised inputs, mean squared error on
log search-node counts, Adam updates, and bfloat16 inference with
round-to-nearest-even at the same points as the GPU kernels.  Parameter block
layout (4553 floats): W1[64][4], b1[64], W2[64][64], b2[64], w3[64], b3,
mu[4], sigma[4].  The analytic gradient here is pinned by central finite
differences of `loss` in the tests.
"""

from __future__ import annotations

import numpy as np

H = 64
_SHAPES = [("W1", (H, 4)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", ()), ("mu", (4,)),
           ("sigma", (4,))]
OFFSETS = {}
_o = 0
for _name, _shape in _SHAPES:
    OFFSETS[_name] = (_o, _shape)
    _o += int(np.prod(_shape)) if _shape else 1
TOTAL = _o
TRAINABLE = OFFSETS["mu"][0]


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out = {}
    for name, (o, shape) in OFFSETS.items():
        size = int(np.prod(shape)) if shape else 1
        out[name] = p[o:o + size].reshape(shape) if shape else p[o]
    return out


def pack(d):
    p = np.zeros(TOTAL, dtype=np.float64)
    for name, (o, shape) in OFFSETS.items():
        size = int(np.prod(shape)) if shape else 1
        p[o:o + size] = np.asarray(d[name], dtype=np.float64).reshape(-1)
    return p


def forward(p, X):
    q = unpack(p)
    Xs = (np.asarray(X, np.float64) - q["mu"]) / q["sigma"]
    a1 = Xs @ q["W1"].T + q["b1"]
    h1 = np.maximum(a1, 0)
    a2 = h1 @ q["W2"].T + q["b2"]
    h2 = np.maximum(a2, 0)
    return h2 @ q["w3"] + q["b3"]


def loss(p, X, t):
    r = forward(p, X) - np.asarray(t, np.float64)
    return float(np.mean(r * r))


def grad(p, X, t):
    """d loss / d p for the trainable block (mu, sigma entries are 0)."""
    q = unpack(p)
    n = len(X)
    Xs = (np.asarray(X, np.float64) - q["mu"]) / q["sigma"]
    a1 = Xs @ q["W1"].T + q["b1"]
    h1 = np.maximum(a1, 0)
    a2 = h1 @ q["W2"].T + q["b2"]
    h2 = np.maximum(a2, 0)
    y = h2 @ q["w3"] + q["b3"]
    dy = 2.0 * (y - np.asarray(t, np.float64)) / n
    g = {k: np.zeros_like(np.asarray(v, np.float64)) for k, v in q.items()}
    g["b3"] = dy.sum()
    g["w3"] = h2.T @ dy
    da2 = np.outer(dy, q["w3"]) * (a2 > 0)
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(0)
    da1 = (da2 @ q["W2"]) * (a1 > 0)
    g["W1"] = da1.T @ Xs
    g["b1"] = da1.sum(0)
    g["mu"] = np.zeros(4)
    g["sigma"] = np.zeros(4)
    return pack(g)


def adam(p, m, v, g, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    p, m, v = p.copy(), m.copy(), v.copy()
    k = slice(0, TRAINABLE)
    m[k] = b1 * m[k] + (1 - b1) * g[k]
    v[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
    mh = m[k] / (1 - b1 ** step)
    vh = v[k] / (1 - b2 ** step)
    p[k] -= lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


def bf16(x):
    """Round float32 values to bfloat16 (nearest, ties to even), as float64."""
    a = np.asarray(x, dtype=np.float32).copy()
    u = a.view(np.uint32).astype(np.uint64)
    nan = np.isnan(a)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    r = (u & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    r[nan] = np.nan
    return r


def forward_bf16(p, X):
    """bfloat16 weights, inputs and hidden activations; products accumulated
    exactly (here in FP64); mu/sigma stay FP32."""
    p32 = np.asarray(p, np.float32)
    pb = bf16(p32)
    pb[TRAINABLE:] = p32[TRAINABLE:]
    q = unpack(pb)
    Xs = bf16(((np.asarray(X, np.float32) - q["mu"].astype(np.float32)) / q["sigma"].astype(np.float32)))
    h1 = bf16(np.maximum(Xs @ q["W1"].T + q["b1"], 0))
    h2 = bf16(np.maximum(h1 @ q["W2"].T + q["b2"], 0))
    return h2 @ q["w3"] + q["b3"]


def init(seed=0):
    """He-style initial weights; identity standardisation."""
    rng = np.random.default_rng(seed)
    d = {"W1": rng.normal(0, np.sqrt(2 / 4), (H, 4)), "b1": np.zeros(H), "W2": rng.normal(0, np.sqrt(2 / H), (H, H)),
         "b2": np.zeros(H), "w3": rng.normal(0, np.sqrt(1 / H), H), "b3": 0.0, "mu": np.zeros(4),
         "sigma": np.ones(4)}
    return pack(d)


def spearman(a, b):
    ra = np.argsort(np.argsort(a, kind="stable"), kind="stable").astype(np.float64)
    rb = np.argsort(np.argsort(b, kind="stable"), kind="stable").astype(np.float64)
    ra -= ra.mean()
    rb -= rb.mean()
    return float((ra * rb).sum() / np.sqrt((ra * ra).sum() * (rb * rb).sum()))
