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
