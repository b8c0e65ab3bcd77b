"""Float64 reference of the learned position model -- test infrastructure only.

The learned model is this project's addition on top of the paper's method (the
paper has no learned component); its definition here is the plain one:

  features   f_k = byte_k / 256 for the 16 address bytes, most significant first
  layer 1    h1 = relu(W1 f + b1)          W1: 64 x 16
  layer 2    h2 = relu(W2 h1 + b2)         W2: 64 x 64
  output     y  = w3 . h2 + b3             w3: 64
  position   p  = clamp(floor(y * m), 0, m - 1)

Parameters are one flat vector in the order W1 (row-major), b1, W2
(row-major), b2, w3, b3 (5,313 values).

Rounding rule (part of the model's definition): a tensor is rounded to
bfloat16 (nearest, ties to even) exactly where it enters a matrix-core product
as an operand.  Forward: the weights W1, W2, w3 and the layer-2 input h1.
Backward: the layer errors dz2 and dz1 where they enter the weight-gradient
products (dz2 also where it is propagated back through W2).  Biases, the
output layer's gradient, the bias gradients and every accumulation stay in
float.  ``rounding=True`` applies these points (the arithmetic in between is
float64); ``rounding=False`` is the exact float64 model.  The rounded path is
pinned against a construction of the same rule from torch's bfloat16
conversion and float64 autograd, with planted misplacements that must differ.

Loss: mean squared error between y and a target; training uses the middle of
the target interval's slot, (i + 1/2) / m, so that floor(y * m) = i.
Optimiser: Adam (Kingma & Ba, 2015) on float32 master weights.
"""
from __future__ import annotations

import numpy as np

H = 64
F = 16
SHAPES = [("W1", (H, F)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)
BF16_PARAMS = ("W1", "W2", "w3")


def unpack(vec):
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = np.asarray(vec[o:o + k], dtype=np.float64).reshape(shape)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16_round(x):
    """Round to the nearest bfloat16, ties to even (via float32, then the top 16 bits)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(f)
    r = np.where(nan, (u | 0x400000) & 0xFFFF0000, r)  # keep NaN a NaN
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def features(addrs):
    """(n, 2) uint64 {hi, lo} -> (n, 16) float64 bytes / 256, MSB first."""
    a = np.asarray(addrs, dtype=np.uint64)
    cols = []
    for word in (a[:, 0], a[:, 1]):
        for k in range(8):
            cols.append(((word >> np.uint64(56 - 8 * k)) & np.uint64(0xFF)).astype(np.float64) / 256.0)
    return np.stack(cols, axis=1)


def model_weights(vec, rounding=True):
    p = unpack(vec)
    if rounding:
        for name in BF16_PARAMS:
            p[name] = bf16_round(p[name])
    return p


def forward(vec, X, rounding=True):
    """Returns y (n,) and the intermediate activations."""
    p = model_weights(vec, rounding)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    h1q = bf16_round(h1) if rounding else h1
    z2 = h1q @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["w3"] + p["b3"][0]
    return y, {"p": p, "X": X, "h1": h1, "h1q": h1q, "h2": h2}


def predict_positions(y, m):
    """p = clamp(floor(y * m), 0, m - 1), with y*m formed in float32 as on the GPU."""
    v = np.floor(np.asarray(y, dtype=np.float32) * np.float32(m)).astype(np.float64)
    return np.clip(v, 0, m - 1).astype(np.int64)


def loss_and_grad(vec, X, t, rounding=True, parts=False):
    """Mean squared error of y against targets t and its gradient w.r.t. vec.
    parts=True also returns the intermediate tensors (for error bounds)."""
    n = X.shape[0]
    y, c = forward(vec, X, rounding)
    p = c["p"]
    r = y - t
    loss = float(np.mean(r * r))
    dy = 2.0 * r / n
    dz2 = np.outer(dy, p["w3"]) * (c["h2"] > 0)
    dz2q = bf16_round(dz2) if rounding else dz2
    g = {}
    g["w3"] = c["h2"].T @ dy
    g["b3"] = np.array([dy.sum()])
    g["b2"] = dz2.sum(axis=0)
    g["W2"] = dz2q.T @ c["h1q"]
    dh1 = dz2q @ p["W2"]
    dz1 = dh1 * (c["h1"] > 0)
    dz1q = bf16_round(dz1) if rounding else dz1
    g["b1"] = dz1.sum(axis=0)
    g["W1"] = dz1q.T @ X
    if parts:
        return loss, pack(g), {"y": y, "dy": dy, "h1q": c["h1q"], "h2": c["h2"], "dz2": dz2, "dz2q": dz2q,
                               "dz1": dz1, "dz1q": dz1q}
    return loss, pack(g)


def adam_step(w, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected); step counts from 1.  Returns (w, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def epsilon_table(pred, idx, m, segments):
    """eps[g] = max |pred_i - idx_i| over the points whose prediction falls in
    segment g = floor(pred * segments / m); segments no point predicts into
    get the marker 2^32 - 1 (search the whole range / fall back)."""
    eps = np.full(segments, 0xFFFFFFFF, dtype=np.uint64)
    seg = (np.asarray(pred, dtype=np.int64) * segments) // m
    err = np.abs(np.asarray(pred, dtype=np.int64) - np.asarray(idx, dtype=np.int64))
    for g, e in zip(seg, err):
        eps[g] = e if eps[g] == 0xFFFFFFFF else max(int(eps[g]), int(e))
    return eps
