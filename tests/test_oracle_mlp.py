"""Pins for the float64 learned-model oracle against independent implementations:
torch's bfloat16 conversion, Python's int.to_bytes, torch CPU float64
autograd and torch.optim.Adam, central finite differences, and a hand-worked
epsilon table."""
import numpy as np
import pytest
import torch

from oracle import mlp

import planb_synth as S


def rand_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(0, scale, mlp.N_PARAMS)


def torch_forward(vec, X):
    v = torch.tensor(vec, dtype=torch.float64, requires_grad=True)
    o, parts = 0, {}
    for name, shape in mlp.SHAPES:
        k = int(np.prod(shape))
        parts[name] = v[o:o + k].reshape(shape)
        o += k
    Xt = torch.tensor(X, dtype=torch.float64)
    h1 = torch.relu(Xt @ parts["W1"].T + parts["b1"])
    h2 = torch.relu(h1 @ parts["W2"].T + parts["b2"])
    return v, h2 @ parts["w3"] + parts["b3"][0]


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 3, 5000), rng.normal(0, 1e-30, 100), [0.0, -0.0, 1.0, 65504.0, 3e38]])
    ties = (rng.integers(0, 2**31, 2000).astype(np.uint32) & 0xFFFF0000) | 0x8000
    x = np.concatenate([x, ties.view(np.float32).astype(np.float64)])
    x = x[np.isfinite(x.astype(np.float32))]
    want = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x), want)


def test_features_are_bytes_over_256():
    a = S.uniform_2000_3(np.random.default_rng(1), 50)
    f = mlp.features(a)
    for i in range(50):
        b = S.to_int(a[i]).to_bytes(16, "big")
        assert list(f[i] * 256) == list(b)


def test_forward_and_gradient_match_torch_autograd():
    vec = rand_params(2)
    X = mlp.features(S.uniform_2000_3(np.random.default_rng(3), 300))
    t = np.random.default_rng(4).random(300)
    y, _ = mlp.forward(vec, X, rounding=False)
    v, yt = torch_forward(vec, X)
    assert np.allclose(y, yt.detach().numpy(), rtol=1e-12, atol=1e-12)
    loss_t = torch.mean((yt - torch.tensor(t)) ** 2)
    loss_t.backward()
    loss, g = mlp.loss_and_grad(vec, X, t, rounding=False)
    assert abs(loss - loss_t.item()) < 1e-12
    assert np.allclose(g, v.grad.numpy(), rtol=1e-10, atol=1e-12)


def test_gradient_matches_finite_differences():
    vec = rand_params(5)
    X = mlp.features(S.uniform_2000_3(np.random.default_rng(6), 64))
    t = np.random.default_rng(7).random(64)
    _, g = mlp.loss_and_grad(vec, X, t, rounding=False)
    rng = np.random.default_rng(8)
    for k in list(rng.integers(0, mlp.N_PARAMS, 40)) + [mlp.N_PARAMS - 1, 0]:
        e = np.zeros_like(vec)
        e[k] = 1e-6
        fd = (mlp.loss_and_grad(vec + e, X, t, False)[0] - mlp.loss_and_grad(vec - e, X, t, False)[0]) / 2e-6
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), k


def test_rounded_gradient_stays_close_to_exact():
    vec = rand_params(9)
    X = mlp.features(S.uniform_2000_3(np.random.default_rng(10), 256))
    t = np.random.default_rng(11).random(256)
    _, g0 = mlp.loss_and_grad(vec, X, t, rounding=False)
    _, g1 = mlp.loss_and_grad(vec, X, t, rounding=True)
    assert np.linalg.norm(g1 - g0) <= 0.05 * np.linalg.norm(g0)


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(12)
    w = rng.normal(size=100)
    wt = torch.tensor(w.copy(), requires_grad=True)
    opt = torch.optim.Adam([wt], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    for step in range(1, 6):
        g = rng.normal(size=100)
        w, m, v = mlp.adam_step(w, m, v, g, step, 1e-3)
        opt.zero_grad()
        wt.grad = torch.tensor(g)
        opt.step()
        assert np.allclose(w, wt.detach().numpy(), rtol=0, atol=1e-12)


def test_epsilon_table_hand_example():
    eps = mlp.epsilon_table([0, 0, 5, 9], [0, 1, 3, 9], 10, 2)
    assert list(eps) == [1, 2]
    eps = mlp.epsilon_table([0, 9], [0, 9], 10, 4)  # segments 1 and 2 get no point
    assert list(eps) == [0, 0xFFFFFFFF, 0xFFFFFFFF, 0]


def test_predicted_positions_clamp():
    assert list(mlp.predict_positions(np.array([-0.5, 0.0, 0.25, 0.9999, 1.7]), 8)) == [0, 0, 2, 7, 7]


def _mutant_no_relu_mask(vec, X, t):
    p = mlp.model_weights(vec, False)
    n = X.shape[0]
    h1 = np.maximum(X @ p["W1"].T + p["b1"], 0)
    h2 = np.maximum(h1 @ p["W2"].T + p["b2"], 0)
    y = h2 @ p["w3"] + p["b3"][0]
    dy = 2 * (y - t) / n
    dz2 = np.outer(dy, p["w3"])  # planted: ReLU mask dropped
    g = {"w3": h2.T @ dy, "b3": np.array([dy.sum()]), "b2": dz2.sum(0), "W2": dz2.T @ h1}
    dz1 = (dz2 @ p["W2"]) * (h1 > 0)
    g["b1"] = dz1.sum(0)
    g["W1"] = dz1.T @ X
    return mlp.pack(g)


def test_planted_gradient_mistake_is_caught():
    vec = rand_params(13, scale=0.6)
    X = mlp.features(S.uniform_2000_3(np.random.default_rng(14), 200))
    t = np.random.default_rng(15).random(200)
    v, yt = torch_forward(vec, X)
    torch.mean((yt - torch.tensor(t)) ** 2).backward()
    assert not np.allclose(_mutant_no_relu_mask(vec, X, t), v.grad.numpy(), rtol=1e-6, atol=1e-9)


# ---------------------------------------------------------------------------
# The bfloat16 rounding path, pinned against an independent construction.
#
# The model's rounding rule, stated once: a tensor is rounded to bfloat16
# exactly where it enters a matrix-core product as an operand -- the weights
# W1, W2 and w3 (stored bf16), the layer-2 input h1 in the forward pass, and,
# in the backward pass, the layer errors dz2 and dz1 that enter the
# weight-gradient products (dz2 also enters the back-propagation product
# dz2 . W2).  Bias gradients, the output layer's gradient and every
# accumulation stay in float.
#
# Below, that rule is written with torch's own bfloat16 conversion and torch
# float64 autograd: QF rounds in the forward pass and is transparent to the
# gradient (weights, h1); QB is the identity forward and rounds the error that
# flows back through it (placed on a layer's matrix product, before its bias
# is added, so the bias gradient sees the unrounded error).  Autograd then
# derives every gradient from the chain rule, with no hand-written backward.
# ---------------------------------------------------------------------------


def _bf16_t(x):
    return x.to(torch.bfloat16).to(torch.float64)


class _QF(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x):
        return _bf16_t(x)

    @staticmethod
    def backward(ctx, g):
        return g


class _QB(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x):
        return x.clone()

    @staticmethod
    def backward(ctx, g):
        return _bf16_t(g)


RULE = dict(w_round=True, h1_round=True, h2_round=False, dz2_round=True, dz1_round=True,
            bias_sees_rounded=False, w3_round=True)


def torch_rounded_loss_and_grad(vec, X, t, **over):
    """Loss, gradient (flat, oracle order) and y of the rounded model built
    from the rule above; keyword overrides plant one misplaced rounding."""
    r = dict(RULE, **over)
    ident = lambda z: z  # noqa: E731
    qf_w = _QF.apply if r["w_round"] else ident
    qb1 = _QB.apply if r["dz1_round"] else ident
    qb2 = _QB.apply if r["dz2_round"] else ident
    v = torch.tensor(vec, dtype=torch.float64, requires_grad=True)
    o, P = 0, {}
    for name, shape in mlp.SHAPES:
        k = int(np.prod(shape))
        P[name] = v[o:o + k].reshape(shape)
        o += k
    Xt = torch.tensor(X, dtype=torch.float64)
    W1, W2 = qf_w(P["W1"]), qf_w(P["W2"])
    w3 = _QF.apply(P["w3"]) if r["w3_round"] else P["w3"]
    if r["bias_sees_rounded"]:
        z1 = qb1(Xt @ W1.T + P["b1"])
    else:
        z1 = qb1(Xt @ W1.T) + P["b1"]
    h1 = torch.relu(z1)
    h1q = _QF.apply(h1) if r["h1_round"] else h1
    if r["bias_sees_rounded"]:
        z2 = qb2(h1q @ W2.T + P["b2"])
    else:
        z2 = qb2(h1q @ W2.T) + P["b2"]
    h2 = torch.relu(z2)
    if r["h2_round"]:
        h2 = _QF.apply(h2)
    y = h2 @ w3 + P["b3"][0]
    loss = torch.mean((y - torch.tensor(t, dtype=torch.float64)) ** 2)
    loss.backward()
    return loss.item(), v.grad.numpy().copy(), y.detach().numpy()


def _rounding_case(seed, n=256):
    vec = rand_params(seed)
    X = mlp.features(S.uniform_2000_3(np.random.default_rng(seed + 1), n))
    t = np.random.default_rng(seed + 2).random(n)
    return vec, X, t


@pytest.mark.parametrize("seed", [21, 22, 23])
def test_rounded_path_matches_independent_construction(seed):
    vec, X, t = _rounding_case(seed)
    loss_t, g_t, y_t = torch_rounded_loss_and_grad(vec, X, t)
    y_o, _ = mlp.forward(vec, X, rounding=True)
    loss_o, g_o = mlp.loss_and_grad(vec, X, t, rounding=True)
    # same rounding decisions on both sides; only float64 summation order differs
    assert np.allclose(y_o, y_t, rtol=1e-12, atol=1e-14)
    assert abs(loss_o - loss_t) <= 1e-12 * max(1.0, abs(loss_t))
    scale = np.abs(g_t).max()
    assert np.allclose(g_o, g_t, rtol=1e-9, atol=1e-12 * scale)


# Each planted mistake moves one rounding point; the oracle must differ from
# it.  (Rounding dz1 before or after the ReLU mask is not among them: the mask
# multiplies by 0 or 1, so the two orders give the same values.)
MUTANTS = {
    "h2 rounded": dict(h2_round=True),
    "h1 not rounded": dict(h1_round=False),
    "dz2 not rounded": dict(dz2_round=False),
    "dz1 not rounded": dict(dz1_round=False),
    "bias gradients from rounded errors": dict(bias_sees_rounded=True),
    "w3 kept in float": dict(w3_round=False),
    "W1/W2 kept in float": dict(w_round=False),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_misplaced_rounding_is_caught(name):
    vec, X, t = _rounding_case(31)
    _, g_o = mlp.loss_and_grad(vec, X, t, rounding=True)
    y_o, _ = mlp.forward(vec, X, rounding=True)
    _, g_m, y_m = torch_rounded_loss_and_grad(vec, X, t, **MUTANTS[name])
    scale = np.abs(g_o).max()
    same_grad = np.allclose(g_o, g_m, rtol=1e-6, atol=1e-9 * scale)
    same_y = np.allclose(y_o, y_m, rtol=1e-9, atol=1e-12)
    assert not (same_grad and same_y), name


@pytest.mark.parametrize("n", [4096, 4096 + 9, 1033])
def test_exact_case_is_exact_in_float32(n):
    """The GPU gradient test's inputs (tests/mlp_exact.py): evaluated in
    float32, in two different summation orders, every decision-feeding
    quantity equals the float64 oracle's exactly, so a float32 kernel takes
    the oracle's rounding and ReLU decisions."""
    from mlp_exact import exact_case
    vec, addrs, t = exact_case(40 + n % 7, n)
    X = mlp.features(addrs)
    _, _, q = mlp.loss_and_grad(vec, X, t.astype(np.float64), parts=True)
    p = mlp.model_weights(vec)
    f32 = {k: v.astype(np.float32) for k, v in p.items()}
    for rev in (False, True):
        order = slice(None, None, -1) if rev else slice(None)

        def mm(a, b):  # float32 products summed one term at a time, in this order
            acc = np.zeros((a.shape[0], b.shape[1]), np.float32)
            for k in range(a.shape[1])[order]:
                acc += a[:, k:k + 1].astype(np.float32) * b[k:k + 1, :].astype(np.float32)
            return acc

        z1 = mm(X.astype(np.float32), f32["W1"].T) + f32["b1"]
        h1q = mlp.bf16_round(np.maximum(z1, 0)).astype(np.float32)
        assert np.array_equal(h1q, q["h1q"])
        z2 = mm(h1q, f32["W2"].T) + f32["b2"]
        h2 = np.maximum(z2, 0)
        assert np.array_equal(h2, q["h2"])
        y = mm(h2, f32["w3"][:, None])[:, 0] + f32["b3"][0]
        assert np.array_equal(y, q["y"])
        dy = (y - t) * np.float32(2.0 / n)
        dz2 = np.where(h2 > 0, dy[:, None] * f32["w3"][None, :], np.float32(0))
        dz2q = mlp.bf16_round(dz2).astype(np.float32)
        assert np.array_equal(dz2q, q["dz2q"])
        dh1 = mm(dz2q, f32["W2"])
        dz1 = np.where(q["h1q"] > 0, dh1, np.float32(0))
        assert np.array_equal(mlp.bf16_round(dz1), q["dz1q"])
