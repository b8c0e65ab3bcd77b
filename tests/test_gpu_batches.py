"""GPU parity of uneven batches in one persistent launch, of its HIP-graph
replays, and of lookups after autotuning -- against the trie oracle."""
import json
import os

import numpy as np
import pytest

import planb_synth as S
from helpers import fib_of, host_u16, oracle_trie, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    from paper_2604_14650_amd import planb
    return planb


def _uneven(fib, sizes, seed):
    addrs = S.zipf_traffic(fib, int(sum(sizes)), seed)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return addrs, offs


def _batches(P, d, out, sizes, offs):
    return [(d[offs[i]:], out[offs[i]:], int(sizes[i])) if sizes[i] else (0, 0, 0) for i in range(len(sizes))]


@pytest.mark.parametrize("kind,seed", [("tiny", 11), ("large", 33)])
def test_persistent_batches_device_descriptors(P, kind, seed):
    import torch
    fib = fib_of(kind, seed)
    rng = np.random.default_rng(5)
    sizes = np.concatenate([[0, 1, 63, 64, 65], S.log_uniform_sizes(rng, 60, 1, 1 << 16), [0]])
    addrs, offs = _uneven(fib, sizes, 77)
    want = oracle_trie(kind, seed).lookup(addrs)
    d = to_dev(addrs)
    out = torch.full((len(addrs),), -1, dtype=torch.int16, device="cuda")
    for fanout in (8, 16, 32):
        h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, fanout=fanout)
        if fanout == 16:  # hybrid descent: binary search in LDS, 2 lanes per lookup below
            P.planb_set_tuning(h, 8, 2, 2, 512, 1)
        arr = P.batch_array(_batches(P, d, out, sizes, offs))
        raw = np.frombuffer(bytes(arr), dtype=np.uint8)
        desc = torch.from_numpy(raw.copy()).cuda()
        for count in (len(sizes), 7):
            say(f"batches {kind} fanout={fanout} count={count}")
            out.fill_(-1)
            cnt = torch.tensor([count], dtype=torch.int32, device="cuda")
            P.planb_lookup_batches(h, desc, cnt, len(sizes))
            got = host_u16(out, len(addrs))
            upto = offs[count]
            assert np.array_equal(got[:upto], want[:upto])
            assert np.all(got[upto:] == 0xFFFF)  # batches beyond the count are untouched


def test_graph_replays_with_changing_batches(P):
    import torch
    fib = fib_of("large", 33)
    want_all = None
    rng = np.random.default_rng(9)
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, fanout=16)
    g = P.Graph(h, 64)
    trie = oracle_trie("large", 33)
    for rep in range(6):
        nb = [64, 13, 1, 0, 40, 64][rep]
        sizes = S.log_uniform_sizes(rng, nb, 1, 1 << 15) if nb else np.zeros(0, np.int64)
        addrs, offs = _uneven(fib, sizes, 100 + rep)
        want = trie.lookup(addrs)
        d = to_dev(addrs) if len(addrs) else None
        out = torch.full((max(1, len(addrs)),), -1, dtype=torch.int16, device="cuda")
        say(f"graph replay {rep} batches={nb} lookups={len(addrs)}")
        g.launch(_batches(P, d, out, sizes, offs) if nb else [])
        # eager work between replays
        eager = torch.full((max(1, len(addrs)),), -1, dtype=torch.int16, device="cuda")
        if len(addrs):
            P.planb_lookup(h, d, len(addrs), eager)
        torch.cuda.synchronize()
        if len(addrs):
            assert np.array_equal(host_u16(out, len(addrs)), want)
            assert np.array_equal(host_u16(eager, len(addrs)), want)
    g.close()


def test_graph_ring_back_to_back(P):
    import torch
    fib = fib_of("tiny", 11)
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops)
    g = P.Graph(h, 8)
    trie = oracle_trie("tiny", 11)
    outs, wants, keep = [], [], []
    for rep in range(11):  # more replays than ring slots, no sync in between
        sizes = np.array([1000 + rep, 7, 4096])
        addrs, offs = _uneven(fib, sizes, 300 + rep)
        d = to_dev(addrs)
        out = torch.full((len(addrs),), -1, dtype=torch.int16, device="cuda")
        g.launch(_batches(P, d, out, sizes, offs))
        outs.append(out)
        keep.append(d)
        wants.append(trie.lookup(addrs))
    torch.cuda.synchronize()
    for out, want in zip(outs, wants):
        assert np.array_equal(host_u16(out, len(want)), want)
    g.close()


def test_graph_rejects_too_many_batches(P):
    fib = fib_of("tiny", 11)
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops)
    g = P.Graph(h, 2)
    with pytest.raises(P.PlanbError) as e:
        g.launch([(0, 0, 0)] * 3)
    assert e.value.code == P.PLANB_ERANGE
    g.close()


def test_autotune_keeps_results_exact(P, tmp_path):
    import torch
    from paper_2604_14650_amd import autotune
    fib = fib_of("backbone", 22)
    addrs = S.backbone_traffic(fib, 1 << 20, seed=4040)
    want = oracle_trie("backbone", 22).lookup(addrs)
    d = to_dev(addrs)
    cache = str(tmp_path / "tune.json")
    h, rec = autotune.tune(fib.prefixes, fib.lengths, fib.next_hops, d, cache_path=cache, reps=1)
    assert not rec["cached"] and rec["fanout"] in (8, 16, 32) and rec["glps"] > 0
    out = torch.empty(len(addrs), dtype=torch.int16, device="cuda")
    P.planb_lookup(h, d, len(addrs), out)
    assert np.array_equal(host_u16(out, len(addrs)), want)
    assert P.planb_get_tuning(h) == rec["tuning"]
    h2, rec2 = autotune.tune(fib.prefixes, fib.lengths, fib.next_hops, d, cache_path=cache)
    assert rec2["cached"] and rec2["fanout"] == rec["fanout"]
    P.planb_lookup(h2, d, len(addrs), out)
    assert np.array_equal(host_u16(out, len(addrs)), want)
    assert json.load(open(cache))


@pytest.mark.parametrize("fanout,key_bits", [(8, 0), (16, 128)])
def test_batches_and_graph_with_key_tops(P, fanout, key_bits):
    """A tuning with lds_search 2: the persistent batch kernel stages the bottom
    internal level as key tops when they fit beside the batch table (else
    whole keys), with 64- and with 128-bit key slots; device descriptors,
    graph replays and eager lookups between them all equal the oracle."""
    import torch
    fib = fib_of("backbone", 22)
    trie = oracle_trie("backbone", 22)
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, fanout=fanout, key_bits=key_bits)
    P.planb_set_tuning(h, fanout // 4, -1, 2, 1024, 2)
    rng = np.random.default_rng(31)
    sizes = np.concatenate([[0, 1, 127, 128, 129], S.log_uniform_sizes(rng, 40, 1, 1 << 17)])
    addrs, offs = _uneven(fib, sizes, 131)
    want = trie.lookup(addrs)
    d = to_dev(addrs)
    out = torch.full((len(addrs),), -1, dtype=torch.int16, device="cuda")
    desc = torch.from_numpy(np.frombuffer(bytes(P.batch_array(_batches(P, d, out, sizes, offs))),
                                          dtype=np.uint8).copy()).cuda()
    cnt = torch.tensor([len(sizes)], dtype=torch.int32, device="cuda")
    say("key tops: device descriptors")
    P.planb_lookup_batches(h, desc, cnt, len(sizes))
    assert np.array_equal(host_u16(out, len(addrs)), want)
    for max_batches in (64, 5000):  # 5000 batch offsets leave no room for the tops: whole keys
        g = P.Graph(h, max_batches)
        for rep in range(3):
            nb = [45, 9, 30][rep]
            sz = S.log_uniform_sizes(rng, nb, 1, 1 << 16)
            a, o = _uneven(fib, sz, 200 + rep)
            w = trie.lookup(a)
            da = to_dev(a)
            go = torch.full((len(a),), -1, dtype=torch.int16, device="cuda")
            say(f"key tops: graph max_batches={max_batches} replay {rep} batches={nb}")
            g.launch(_batches(P, da, go, sz, o))
            eager = torch.full((len(a),), -1, dtype=torch.int16, device="cuda")
            P.planb_lookup(h, da, len(a), eager)
            torch.cuda.synchronize()
            assert np.array_equal(host_u16(go, len(a)), w)
            assert np.array_equal(host_u16(eager, len(a)), w)
        g.close()


def test_uneven_batches_up_to_4m_on_the_large_fib(P):
    """The 1M-prefix FIB with /128 host routes (128-bit keys) and Zipf(1.1)
    batches of 64 .. 2^22 addresses, with launch shapes autotuned per batch-size
    bucket: planb_lookup per batch (each taking its bucket's shape), one
    persistent launch over every batch, and graph replays (every batch in one
    replay, and batches one at a time through a graph of the smallest bucket's
    shape) all equal the oracle."""
    import torch
    from paper_2604_14650_amd import autotune
    fib = fib_of("large", 33)
    rng = np.random.default_rng(41)
    sizes = np.concatenate([[64, 65, 4097, (1 << 20) + 3, 1 << 22], S.log_uniform_sizes(rng, 27, 64, 1 << 22)])
    addrs, offs = _uneven(fib, sizes, 1033)
    want = oracle_trie("large", 33).lookup(addrs)
    d = to_dev(addrs)
    buckets = [256, 4096, 1 << 16, 1 << 20, 1 << 22]
    say(f"large FIB: {len(sizes)} batches, {len(addrs)} lookups; autotuning {buckets}")
    h, rec = autotune.tune_sizes(fib.prefixes, fib.lengths, fib.next_hops, d, buckets, fanouts=(16,),
                                 cache_path=None, reps=1)
    assert P.planb_get_info(h)["key_bits"] == 128
    table = P.planb_get_size_tunings(h)
    assert [e[0] for e in table] == [e["min_lookups"] for e in rec["buckets"]] and table[0][0] == 1
    out = torch.full((len(addrs),), -1, dtype=torch.int16, device="cuda")
    say("per-batch planb_lookup with the bucket shapes")
    for i, m in enumerate(sizes):
        P.planb_lookup(h, d[offs[i]:], int(m), out[offs[i]:])
    assert np.array_equal(host_u16(out, len(addrs)), want)
    say("one persistent launch over every batch")
    out.fill_(-1)
    desc = torch.from_numpy(np.frombuffer(bytes(P.batch_array(_batches(P, d, out, sizes, offs))),
                                          dtype=np.uint8).copy()).cuda()
    cnt = torch.tensor([len(sizes)], dtype=torch.int32, device="cuda")
    P.planb_lookup_batches(h, desc, cnt, len(sizes))
    assert np.array_equal(host_u16(out, len(addrs)), want)
    say("the persistent launch's shape chosen by timing this batch set")
    cands = [table[-1][1], table[-2][1], table[0][1]]
    shape, ms = autotune.tune_batches(h, desc, cnt, len(sizes), cands, reps=1)
    assert shape in cands and sorted(ms) == list(range(len(cands)))
    assert P.planb_get_tuning(h) == shape
    out.fill_(-1)
    P.planb_lookup_batches(h, desc, cnt, len(sizes))
    assert np.array_equal(host_u16(out, len(addrs)), want)
    say("every batch in one graph replay")
    g = P.Graph(h, 64)
    out.fill_(-1)
    g.launch(_batches(P, d, out, sizes, offs))
    torch.cuda.synchronize()
    assert np.array_equal(host_u16(out, len(addrs)), want)
    g.close()
    P.planb_set_tuning(h, **table[0][1])
    g = P.Graph(h, 4)
    out.fill_(-1)
    for i in range(len(sizes)):
        say(f"single-batch graph replay {i}, {int(sizes[i])} lookups")
        g.launch([(d[offs[i]:], out[offs[i]:], int(sizes[i]))])
    torch.cuda.synchronize()
    assert np.array_equal(host_u16(out, len(addrs)), want)
    g.close()
    P.planb_set_size_tunings(h, [])
    assert P.planb_get_size_tunings(h) == []


def test_size_tunings_are_checked(P):
    fib = fib_of("tiny", 11)
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, fanout=16)
    good = P.planb_get_tuning(h)
    with pytest.raises(P.PlanbError) as e:
        P.planb_set_size_tunings(h, [(100, good), (100, good)])
    assert e.value.code == P.PLANB_EINVAL
    bad = dict(good, keys_per_lane=3)
    with pytest.raises(P.PlanbError):
        P.planb_set_size_tunings(h, [(1, good), (1000, bad)])
    assert P.planb_get_size_tunings(h) == []  # unchanged on error
    P.planb_set_size_tunings(h, [(1, good), (1000, dict(good, lookups_per_group=1))])
    assert [e[0] for e in P.planb_get_size_tunings(h)] == [1, 1000]
