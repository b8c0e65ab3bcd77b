"""Inputs on which the learned model's float32 kernels must agree with the
float64 oracle element by element (test infrastructure, no method arithmetic
beyond calls into oracle/mlp.py).

The parameters are small dyadic rationals and the address bytes multiples of
16, so that every quantity that feeds a decision -- a ReLU mask, a bfloat16
rounding of h1, dz2 or dz1, the output y -- is computed exactly in float32
whatever the summation order (each is a sum of terms on a fixed power-of-two
grid whose absolute sum stays below 2^24 grid steps).  Both sides then take
the same rounding and mask decisions, and the gradient differs from the
oracle's only by the float32 accumulation of its final sums over samples:

    |g_gpu - g_oracle| <= (2n + 2) * 2^-24 * A  (+ 2^-21 * A for a batch size
                          that is not a power of two)

element by element, where A is the same sum taken over absolute values.

With a batch size n that is not a power of two the kernel's 2/n is rounded to
float32, which perturbs every dy and dz2 by a relative 2^-23 at most; each
sample's single dz2 magnitude (|w3| is 1/16 for every unit) is then kept more
than that away from a bfloat16 rounding midpoint by re-drawing its target.
"""
from __future__ import annotations

import numpy as np

from oracle import mlp


def dyadic_params(seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    p = mlp.unpack(np.zeros(mlp.N_PARAMS))
    p["W1"] = rng.integers(-16, 17, (64, 16)) / 32.0        # grid 2^-5, |w| <= 1/2
    p["b1"] = rng.integers(-64, 65, 64) / 2.0 ** 9          # grid 2^-9
    p["W2"] = rng.integers(-8, 9, (64, 64)) / 32.0          # grid 2^-5, |w| <= 1/4
    p["b2"] = rng.integers(-2048, 2049, 64) / 2.0 ** 14     # grid 2^-14
    p["w3"] = rng.choice([-1.0, 1.0], 64) / 16.0
    p["b3"] = np.array([rng.integers(0, 2 ** 19) / 2.0 ** 20])
    return mlp.pack(p)


def coarse_addresses(seed: int, n: int) -> np.ndarray:
    """(n, 2) uint64 addresses whose 16 bytes are multiples of 16."""
    rng = np.random.default_rng(seed)
    b = (rng.integers(0, 16, (n, 16)) * 16).astype(np.uint64)
    hi = np.zeros(n, np.uint64)
    lo = np.zeros(n, np.uint64)
    for k in range(8):
        hi |= b[:, k] << np.uint64(56 - 8 * k)
        lo |= b[:, 8 + k] << np.uint64(56 - 8 * k)
    return np.stack([hi, lo], axis=1)


def _near_bf16_midpoint(v: np.ndarray, rel: float) -> np.ndarray:
    """True where v (> 0) lies within a relative `rel` of a point halfway
    between two neighbouring bfloat16 values."""
    e = np.floor(np.log2(v))
    units = v / 2.0 ** (e - 7)          # v in bf16 steps of its binade, in [128, 256)
    frac = units - np.floor(units)
    return np.abs(frac - 0.5) * 2.0 ** (e - 7) <= rel * v


def exact_case(seed: int, n: int):
    """(params, addresses, float32 targets) for a gradient test of n samples."""
    vec = dyadic_params(seed)
    addrs = coarse_addresses(seed + 1, n)
    X = mlp.features(addrs)
    y, c = mlp.forward(vec, X)
    rng = np.random.default_rng(seed + 2)
    pow2 = (n & (n - 1)) == 0
    delta = np.empty(n)
    todo = np.ones(n, bool)
    while todo.any():
        k = int(todo.sum())
        d = (0.25 + rng.integers(0, 2 ** 18, k) / 2.0 ** 20) * rng.choice([-1.0, 1.0], k)
        delta[todo] = d
        if pow2:
            break
        bad = _near_bf16_midpoint(np.abs(2.0 * delta / n / 16.0), 2.0 ** -21)
        todo = bad
    t = y - delta                                            # on the 2^-20 grid
    # exactness budgets (float32 has a 24-bit significand)
    assert np.all(np.abs(c["h2"]) @ np.full(64, 1 / 16.0) + abs(mlp.unpack(vec)["b3"][0]) < 16.0)
    assert np.all(np.abs(t) < 16.0)
    assert np.array_equal(t.astype(np.float32).astype(np.float64), t)
    return vec, addrs, t.astype(np.float32)


def grad_bound(vec, addrs, t) -> tuple[np.ndarray, np.ndarray]:
    """The oracle's gradient and its element-wise float32 bound (see above)."""
    n = addrs.shape[0]
    X = mlp.features(addrs)
    _, g, q = mlp.loss_and_grad(vec, X, t.astype(np.float64), parts=True)
    A = mlp.pack({
        "W1": np.abs(q["dz1q"]).T @ np.abs(X),
        "b1": np.abs(q["dz1"]).sum(axis=0),
        "W2": np.abs(q["dz2q"]).T @ np.abs(q["h1q"]),
        "b2": np.abs(q["dz2"]).sum(axis=0),
        "w3": np.abs(q["h2"]).T @ np.abs(q["dy"]),
        "b3": np.array([np.abs(q["dy"]).sum()]),
    })
    pow2 = (n & (n - 1)) == 0
    bound = (2 * n + 2) * 2.0 ** -24 * A + (0.0 if pow2 else 2.0 ** -21 * A)
    return g, bound
