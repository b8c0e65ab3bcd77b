"""IPv4 on the GPU: FIBs of rules of at most /32 in the top 32 bits get 32-bit
key slots; lookups through 16-byte records and through 4-byte addresses
(planb_lookup_v4) must equal the oracle's next hops."""
import functools

import numpy as np
import pytest

import planb_synth as S
from helpers import host_u16, out_u16, say, to_dev
from oracle.brute import lpm_bruteforce
from oracle.trie import Trie

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    from paper_2604_14650_amd import planb
    return planb


@functools.lru_cache(maxsize=None)
def _fib(kind, seed):
    return S.make_fib({"tiny": S.IPV4_TINY, "full": S.IPV4}[kind], seed)


@functools.lru_cache(maxsize=None)
def _trie(kind, seed):
    f = _fib(kind, seed)
    return Trie(f.prefixes, f.lengths, f.next_hops)


def _v4_dev(a4):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a4).view(np.int32)).cuda()


def _both(P, h, a4):
    """Next hops through 16-byte records and through 4-byte addresses."""
    n = a4.shape[0]
    o1 = out_u16(n)
    P.planb_lookup(h, to_dev(S.v4_as_128(a4)), n, o1)
    o2 = out_u16(n)
    P.planb_lookup_v4(h, _v4_dev(a4), n, o2)
    return host_u16(o1, n), host_u16(o2, n)


VARIANTS = [(8, 1, 1, 0), (8, 2, 2, 0), (8, 8, 2, 0), (16, 4, 2, 0), (16, 16, 1, 0), (32, 1, 1, 0), (32, 8, 4, 0),
            (8, 8, 1, 1), (8, 2, 2, 1), (16, 4, 4, 1), (16, 8, 2, 1), (32, 16, 2, 1), (32, 8, 1, 1)]


@pytest.mark.parametrize("fanout,kpl,R,bin_", VARIANTS)
def test_tiny_ipv4_all_variants(P, fanout, kpl, R, bin_):
    fib = _fib("tiny", 1)
    a4 = S.ipv4_traffic(fib, 1 << 18, 0.6, 11)
    a4 = np.concatenate([a4, np.array([0, 1, 0xFFFFFFFF, 0xFFFFFFFE, 0x80000000], np.uint32)])
    want = _trie("tiny", 1).lookup(S.v4_as_128(a4))
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, fanout=fanout)
    info = P.planb_get_info(h)
    assert info["key_bits"] == 32 and info["leaf_keys"] == 20 and info["leaf_slots"] == 32
    depth = info["depth"]
    for lds, block in sorted({(0, 512), (-1, 512), (depth, 1024), (max(0, depth - 1), 512)}):
        say(f"ipv4 tiny fanout={fanout} kpl={kpl} R={R} bin={bin_} lds={lds} block={block}")
        try:
            P.planb_set_tuning(h, kpl, lds, R, block, bin_)
        except P.PlanbError:
            continue  # more levels than fit in LDS
        g16, g4 = _both(P, h, a4)
        assert np.array_equal(g16, want)
        assert np.array_equal(g4, want)


@pytest.mark.parametrize("fanout", [8, 16, 32])
def test_full_ipv4_table(P, fanout):
    fib = _fib("full", 5)
    a4 = S.ipv4_traffic(fib, 1 << 22, 0.7, 12)
    want = _trie("full", 5).lookup(S.v4_as_128(a4))
    say(f"ipv4 full fanout={fanout}")
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, fanout=fanout)
    assert P.planb_get_info(h)["key_bits"] == 32
    g16, g4 = _both(P, h, a4)
    assert np.array_equal(g16, want) and np.array_equal(g4, want)
    # the same FIB with 64- and 128-bit slots gives the same answers
    for kb in (64, 128):
        h2 = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, fanout=fanout, key_bits=kb)
        o = out_u16(a4.shape[0])
        P.planb_lookup(h2, to_dev(S.v4_as_128(a4)), a4.shape[0], o)
        assert np.array_equal(host_u16(o, a4.shape[0]), want), kb


def test_ipv4_edge_rules(P):
    top = lambda v: v << 96  # noqa: E731
    rules = [(0, 0, 1), (top(0xFFFFFFFF), 32, 2), (top(0xFF000000), 8, 3), (0, 32, 4), (top(0x0A000000), 8, 5),
             (top(0x0A010000), 16, 6), (top(0x0A010100), 24, 7), (top(0x0A010101), 32, 8)]
    p = S.from_ints([r[0] for r in rules])
    L = np.array([r[1] for r in rules], np.uint8)
    nh = np.array([r[2] for r in rules], np.uint16)
    a4 = np.array(sorted({0, 1, 0xFFFFFFFF, 0xFFFFFFFE, 0xFF000000, 0xFEFFFFFF, 0x0A000000, 0x09FFFFFF,
                          0x0A010100, 0x0A0100FF, 0x0A010101, 0x0A010102, 0x0AFFFFFF, 0x0B000000}), np.uint32)
    want = lpm_bruteforce(p, L, nh, S.v4_as_128(a4))
    for fanout in (8, 16, 32):
        h = P.planb_build(p, L, nh, fanout=fanout)
        assert P.planb_get_info(h)["key_bits"] == 32
        for kpl, lds, bin_ in ((1, 0, 0), (fanout, -1, 1), (fanout // 2, 1, 1)):
            P.planb_set_tuning(h, kpl, lds, 2, 512, bin_)
            g16, g4 = _both(P, h, a4)
            assert np.array_equal(g16, want) and np.array_equal(g4, want), (fanout, kpl, lds, bin_)


def test_v4_entry_refuses_wider_keys(P):
    fib = _fib("tiny", 1)
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, key_bits=64)
    with pytest.raises(P.PlanbError) as e:
        P.planb_lookup_v4(h, _v4_dev(np.zeros(4, np.uint32)), 4, out_u16(4))
    assert e.value.code == P.PLANB_EINVAL


def test_ipv4_device_build_and_learned(P):
    import torch
    fib = _fib("full", 5)
    host = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, fanout=16)
    dp = torch.from_numpy(np.ascontiguousarray(fib.prefixes).view(np.int64)).cuda()
    dL = torch.from_numpy(np.ascontiguousarray(fib.lengths)).cuda()
    dn = torch.from_numpy(np.ascontiguousarray(fib.next_hops).view(np.int16)).cuda()
    dev = P.planb_build_device(dp, dL, dn, fanout=16)
    assert P.planb_get_info(dev)["key_bits"] == 32
    assert np.array_equal(P.planb_export_image(host), P.planb_export_image(dev))
    a4 = S.ipv4_traffic(fib, 1 << 20, 0.7, 13)
    want = _trie("full", 5).lookup(S.v4_as_128(a4))
    P.planb_train(dev, seed=3)
    o = out_u16(a4.shape[0])
    P.planb_lookup_learned(dev, to_dev(S.v4_as_128(a4)), a4.shape[0], o)
    assert np.array_equal(host_u16(o, a4.shape[0]), want)
    m = 1 << 16  # a small call: the queue-free kernel, fallbacks descended in place
    o2 = out_u16(m)
    P.planb_lookup_learned(dev, to_dev(S.v4_as_128(a4[:m])), m, o2)
    assert np.array_equal(host_u16(o2, m), want[:m])


def test_ipv4_batches_and_multi(P):
    import torch
    tabs = [_fib("tiny", s) for s in (1, 2, 3)]
    tries = [_trie("tiny", s) for s in (1, 2, 3)]
    ts = P.TableSet(4)
    fibs = [P.planb_build(t.prefixes, t.lengths, t.next_hops, fanout=16) for t in tabs]
    for k, f in enumerate(fibs):
        ts.set(k, f)
    rng = np.random.default_rng(4)
    sizes = [int(x) for x in rng.integers(1, 3000, size=30)]
    tids = rng.integers(0, 3, size=30)
    addrs = [S.v4_as_128(S.ipv4_traffic(tabs[t], n, 0.6, int(rng.integers(0, 2**31)))) for t, n in zip(tids, sizes)]
    flat = np.concatenate(addrs)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    d = to_dev(flat)
    out = torch.full((len(flat),), -1, dtype=torch.int16, device="cuda")
    rows = [(int(tids[i]), d[offs[i]:], out[offs[i]:], sizes[i]) for i in range(len(sizes))]
    desc = torch.from_numpy(np.frombuffer(bytes(P.burst_array(rows)), dtype=np.uint8).copy()).cuda()
    cnt = torch.tensor([len(rows)], dtype=torch.int32, device="cuda")
    P.planb_lookup_multi(ts, desc, cnt, len(rows))
    got = host_u16(out, len(flat))
    for i in range(len(sizes)):
        assert np.array_equal(got[offs[i]:offs[i + 1]], tries[tids[i]].lookup(addrs[i])), i
    # persistent batches on one IPv4 FIB
    h = fibs[0]
    bsz = [1, 63, 64, 65, 5000, 77777]
    a = S.v4_as_128(S.ipv4_traffic(tabs[0], sum(bsz), 0.6, 9))
    want = tries[0].lookup(a)
    da = to_dev(a)
    o = torch.full((len(a),), -1, dtype=torch.int16, device="cuda")
    bo = np.concatenate([[0], np.cumsum(bsz)]).astype(np.int64)
    g = P.Graph(h, len(bsz))
    g.launch([(da[bo[i]:], o[bo[i]:], bsz[i]) for i in range(len(bsz))])
    torch.cuda.synchronize()
    assert np.array_equal(host_u16(o, len(a)), want)
    g.close()
