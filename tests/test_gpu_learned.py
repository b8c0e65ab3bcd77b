"""Learned position model on the GPU, through the C ABI:

* inference, gradient and Adam kernels against the float64 oracle
  (oracle/mlp.py) on the same seeded parameters and samples;
* training is deterministic and its error table bounds every boundary point;
* learned lookups are bit-exact against the LPM oracle, also with the window
  search forced to fail (zero or empty error bounds) and with random weights.
"""
import numpy as np
import pytest

import planb_synth as S
from helpers import fib_of, host_u16, oracle_trie, say, to_dev
from oracle import mlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    from paper_2604_14650_amd import planb
    return planb


def seeded_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    p = mlp.unpack(np.zeros(mlp.N_PARAMS))
    p["W1"] = rng.uniform(-0.25, 0.25, (64, 16)) * scale
    p["b1"] = rng.normal(0, 0.05, 64)
    p["W2"] = rng.uniform(-0.125, 0.125, (64, 64)) * scale
    p["b2"] = rng.normal(0, 0.05, 64)
    p["w3"] = rng.uniform(-0.125, 0.125, 64)
    p["b3"] = np.array([0.5])
    return mlp.pack(p).astype(np.float32).astype(np.float64)


def f32_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _magnitude(vec, X):
    """S(x) = sum_u |w3_u| sum_v |W2_uv| |h1_v| : scale of y's sensitivity to h1."""
    p = mlp.model_weights(vec)
    _, c = mlp.forward(vec, X)
    return (np.abs(c["h1q"]) @ np.abs(p["W2"]).T) @ np.abs(p["w3"]) + np.abs(p["b3"][0])


def test_predict_matches_oracle(P):
    import torch
    fib = fib_of("tiny", 11)
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops)
    vec = seeded_params(1)
    P.planb_model_set_params(h, vec)
    addrs = S.tiny_traffic(fib, 1 << 14, seed=9)
    y = torch.empty(len(addrs), dtype=torch.float32, device="cuda")
    P.planb_model_predict(h, to_dev(addrs), len(addrs), y)
    got = y.cpu().numpy().astype(np.float64)
    X = mlp.features(addrs)
    want, _ = mlp.forward(vec, X)
    Sx = _magnitude(vec, X)
    err = np.abs(got - want)
    # float32 accumulation plus at most one flipped bf16 rounding per h1 element
    assert np.all(err <= 2.0 ** -8 * Sx + 1e-6), err.max()
    assert np.median(err / Sx) < 1e-5


@pytest.mark.parametrize("n", [4096, 4096 + 9, 1033, 1 << 15])
def test_gradient_matches_oracle_elementwise(P, n):
    """Every gradient entry within its float32 accumulation bound of the
    float64 oracle, on inputs where both sides take the same rounding and
    ReLU decisions (tests/mlp_exact.py): one tile, ragged tails, and more
    tiles than the kernel's grid holds."""
    import torch
    from mlp_exact import exact_case, grad_bound
    fib = fib_of("tiny", 11)
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops)
    vec, samples, t = exact_case(40 + n % 7, n)
    P.planb_model_set_params(h, vec)
    say(f"gradient parity n={n}")
    g = torch.empty(mlp.N_PARAMS, dtype=torch.float32, device="cuda")
    P.planb_model_grad(h, to_dev(samples), f32_dev(t), n, g)
    got = g.cpu().numpy().astype(np.float64)
    want, bound = grad_bound(vec, samples, t)
    err = np.abs(got - want)
    worst = int(np.argmax(err - bound))
    assert np.all(err <= bound), (worst, got[worst], want[worst], bound[worst])


def test_predict_exact_on_dyadic_model(P):
    """With exactly representable parameters and inputs the forward pass is
    exact in float32, so y must equal the oracle's bit for bit."""
    import torch
    from mlp_exact import coarse_addresses, dyadic_params
    fib = fib_of("tiny", 11)
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops)
    vec = dyadic_params(50)
    P.planb_model_set_params(h, vec)
    addrs = coarse_addresses(51, 5000 + 3)
    y = torch.empty(len(addrs), dtype=torch.float32, device="cuda")
    P.planb_model_predict(h, to_dev(addrs), len(addrs), y)
    want, _ = mlp.forward(vec, mlp.features(addrs))
    assert np.array_equal(y.cpu().numpy().astype(np.float64), want)


def test_adam_matches_oracle(P):
    import torch
    fib = fib_of("tiny", 11)
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops)
    vec = seeded_params(4)
    P.planb_model_set_params(h, vec)
    rng = np.random.default_rng(5)
    w = vec.copy()
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    for step in range(1, 5):
        grad = rng.normal(0, 1e-2, mlp.N_PARAMS).astype(np.float32)
        P.planb_model_adam(h, f32_dev(grad), 1e-3)
        w, m, v = mlp.adam_step(w, m, v, grad.astype(np.float64), step, 1e-3)
    torch.cuda.synchronize()
    got = P.planb_model_get_params(h).astype(np.float64)
    assert np.max(np.abs(got - w)) < 2e-6


@pytest.fixture(scope="module")
def trained_tiny(P):
    fib = fib_of("tiny", 11)
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops)
    rep = P.planb_train(h, seed=7)
    say(f"tiny training report {rep}")
    return fib, h, rep


def test_training_is_deterministic(P, trained_tiny):
    fib, h, rep = trained_tiny
    h2 = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops)
    rep2 = P.planb_train(h2, seed=7)
    assert np.array_equal(P.planb_model_get_params(h), P.planb_model_get_params(h2))
    assert np.array_equal(P.planb_model_get_eps(h, 4096), P.planb_model_get_eps(h2, 4096))
    assert rep["final_loss"] == rep2["final_loss"]


def test_training_reduces_loss(P, trained_tiny):
    import torch
    fib, h, rep = trained_tiny
    starts, _ = P.planb_export_intervals(h)
    m = len(starts)
    t = (np.arange(m) + 0.5) / m
    y = torch.empty(m, dtype=torch.float32, device="cuda")
    P.planb_model_predict(h, to_dev(starts), m, y)
    loss = np.mean((y.cpu().numpy() - t) ** 2)
    # far below the best constant predictor's loss (the variance of t)
    assert loss < 0.01 * np.var(t)
    assert rep["steps"] >= 1000 and rep["max_eps"] < m // 4


def test_error_table_bounds_every_boundary_point(P, trained_tiny):
    import torch
    fib, h, rep = trained_tiny
    starts, _ = P.planb_export_intervals(h)
    m = len(starts)
    ints = [S.to_int(r) for r in starts]
    lasts = [(ints[i + 1] - 1) if i + 1 < m else (1 << 128) - 1 for i in range(m)]
    pts = np.concatenate([starts, S.from_ints(lasts)])
    idx = np.concatenate([np.arange(m)] * 2)
    y = torch.empty(len(pts), dtype=torch.float32, device="cuda")
    P.planb_model_predict(h, to_dev(pts), len(pts), y)
    p = mlp.predict_positions(y.cpu().numpy(), m)
    eps = P.planb_model_get_eps(h, 4096).astype(np.int64)
    assert len(eps) == max(1, min(4096, m // 64))  # at least 64 positions per segment
    seg = p * len(eps) // m
    assert np.all(eps[seg] != 0xFFFFFFFF)
    assert np.all(np.abs(p - idx) <= eps[seg])


def test_prediction_error_on_traffic_is_near_the_table(P, trained_tiny):
    """Lookup traffic (random low bytes) is predicted about as well as the
    table's points: most addresses land inside their widened window."""
    import torch
    fib, h, rep = trained_tiny
    addrs = S.tiny_traffic(fib, 1 << 15, seed=21)
    d = to_dev(addrs)
    y = torch.empty(len(addrs), dtype=torch.float32, device="cuda")
    P.planb_model_predict(h, d, len(addrs), y)
    idx = torch.empty(len(addrs), dtype=torch.int32, device="cuda")
    P.planb_lookup_index(h, d, len(addrs), idx)
    m = P.planb_num_intervals(h)
    p = mlp.predict_positions(y.cpu().numpy(), m)
    eps = P.planb_model_get_eps(h, 4096).astype(np.int64)
    e = eps[p * len(eps) // m]
    inside = np.abs(p - idx.cpu().numpy()) <= e + e // 2 + 16
    assert inside.mean() > 0.9


def _learned(P, h, addrs):
    import torch
    d = to_dev(addrs)
    out = torch.full((len(addrs),), -1, dtype=torch.int16, device="cuda")
    fb = torch.zeros(1, dtype=torch.int32, device="cuda")
    P.planb_lookup_learned(h, d, len(addrs), out, fb)
    return host_u16(out, len(addrs)), int(fb.item())


def test_learned_lookup_exact_tiny(P, trained_tiny):
    fib, h, rep = trained_tiny
    addrs = S.tiny_traffic(fib, 1 << 20, seed=1011)
    want = oracle_trie("tiny", 11).lookup(addrs)
    got, fb = _learned(P, h, addrs)
    say(f"tiny learned fallbacks {fb} of {len(addrs)}")
    assert np.array_equal(got, want)
    assert fb < 0.05 * len(addrs)


@pytest.mark.parametrize("key_bits", [0, 128])
def test_learned_lookup_ragged_sizes(P, key_bits):
    """Batches of 0, 1, 63, 64, 65, 1000, 4097 and 12345 addresses, through the
    leaf-tops kernel (64-bit key slots) and the subtree search (128-bit): every
    result equals the oracle's and nothing past n is written."""
    import torch
    fib = fib_of("tiny", 11)
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, key_bits=key_bits)
    P.planb_train(h, seed=5)
    addrs = S.tiny_traffic(fib, 12345, seed=77)
    want = oracle_trie("tiny", 11).lookup(addrs)
    d = to_dev(addrs)
    for n in (0, 1, 63, 64, 65, 1000, 4097, 12345):
        say(f"learned ragged key_bits={key_bits} n={n}")
        out = torch.full((len(addrs) + 64,), -1, dtype=torch.int16, device="cuda")
        P.planb_lookup_learned(h, d, n, out)
        got = host_u16(out, len(addrs) + 64)
        assert np.array_equal(got[:n], want[:n]), n
        assert np.all(got[n:] == 0xFFFF), n


@pytest.mark.parametrize("n", [1 << 16, (1 << 21) + 5])
@pytest.mark.parametrize("key_bits", [0, 128])
def test_forced_fallbacks_stay_exact(P, key_bits, n):
    """Error bounds forced to zero (windows of a few positions), to "empty" and
    to the whole range.  With 64-bit key slots the leaf-tops kernel runs, with
    128-bit slots the subtree search; in both an empty segment searches the
    whole tree (no fallback).  2^16 lookups run the direct kernel (failing
    lookups descend in place), 2^21 + 5 the queued one (a fallback kernel
    descends them).  Every result equals the oracle's."""
    fib = fib_of("tiny", 11)
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, key_bits=key_bits)
    P.planb_train(h, seed=7)
    addrs = S.tiny_traffic(fib, n, seed=12)
    want = oracle_trie("tiny", 11).lookup(addrs)
    G = len(P.planb_model_get_eps(h, 4096))
    P.planb_model_set_eps(h, np.zeros(G, np.uint32))  # windows of +-16 positions only
    got, fb = _learned(P, h, addrs)
    assert np.array_equal(got, want) and fb > 0
    P.planb_model_set_eps(h, np.full(G, 0xFFFFFFFF, np.uint32))
    got, fb = _learned(P, h, addrs)
    assert np.array_equal(got, want) and fb == 0
    P.planb_model_set_eps(h, np.full(G, 1 << 30, np.uint32))  # whole-range windows
    got, fb = _learned(P, h, addrs)
    assert np.array_equal(got, want) and fb == 0


def _interval_edges(fib):
    """Every prefix's first and last address and their outer neighbours, plus
    the two ends of the address space: the addresses where one interval ends
    and the next begins (computed from the rules alone, as 128-bit integers)."""
    pts = {0, (1 << 128) - 1}
    for (hi, lo), ln in zip(fib.prefixes.tolist(), fib.lengths.tolist()):
        span = 1 << (128 - ln)
        a = ((hi << 64) | lo) & ~(span - 1)
        for v in (a - 1, a, a + span - 1, a + span):
            if 0 <= v < (1 << 128):
                pts.add(v)
    v = sorted(pts)
    return np.array([[x >> 64, x & ((1 << 64) - 1)] for x in v], dtype=np.uint64)


@pytest.mark.parametrize("key_bits", [0, 128])
def test_mixed_windows_at_interval_edges(P, key_bits):
    """Error bounds that differ wildly from segment to segment (zero, small,
    large, beyond the table, "empty"), so that one wavefront's lanes search
    windows of very different widths with the same steps, on addresses at every
    interval edge of the FIB and at both ends of the address space.  Every
    result equals the oracle's."""
    fib = fib_of("tiny", 11)
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, key_bits=key_bits)
    P.planb_train(h, seed=9)
    edges = _interval_edges(fib)
    rng = np.random.default_rng(31)
    addrs = np.concatenate([edges, S.tiny_traffic(fib, 1 << 14, seed=14)])
    addrs = addrs[rng.permutation(len(addrs))]
    want = oracle_trie("tiny", 11).lookup(addrs)
    G = len(P.planb_model_get_eps(h, 4096))
    for trial in range(3):
        eps = rng.choice(np.array([0, 3, 40, 700, 1 << 20, 0xFFFFFFFF], dtype=np.uint32), size=G)
        P.planb_model_set_eps(h, eps)
        got, fb = _learned(P, h, addrs)
        say(f"mixed windows key_bits={key_bits} trial {trial}: {len(addrs)} addresses, {fb} fallbacks")
        assert np.array_equal(got, want), trial


def test_random_weights_stay_exact(P):
    fib = fib_of("tiny", 11)
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, fanout=8)
    P.planb_model_set_params(h, seeded_params(21, scale=3.0), 256)
    P.planb_model_build_eps(h)
    addrs = S.tiny_traffic(fib, 1 << 16, seed=13)
    got, _ = _learned(P, h, addrs)
    assert np.array_equal(got, oracle_trie("tiny", 11).lookup(addrs))


@pytest.mark.parametrize("kind,seed,fanout", [("backbone", 22, 8), ("backbone", 22, 16), ("large", 33, 16)])
def test_learned_lookup_exact_large_fibs(P, kind, seed, fanout):
    fib = fib_of(kind, seed)
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, fanout=fanout)
    rep = P.planb_train(h, seed=3)
    say(f"{kind} fanout={fanout} training report {rep}")
    addrs = S.backbone_traffic(fib, 1 << 21, seed=2222) if kind == "backbone" else S.zipf_traffic(fib, 1 << 21, 7)
    want = oracle_trie(kind, seed).lookup(addrs)
    got, fb = _learned(P, h, addrs)
    say(f"{kind} learned fallbacks {fb} of {len(addrs)}")
    assert np.array_equal(got, want)


def test_learned_requires_a_model(P):
    import torch
    fib = fib_of("tiny", 11)
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops)
    d = to_dev(S.tiny_traffic(fib, 64, seed=1))
    out = torch.empty(64, dtype=torch.int16, device="cuda")
    with pytest.raises(P.PlanbError) as e:
        P.planb_lookup_learned(h, d, 64, out)
    assert e.value.code == P.PLANB_EINVAL
