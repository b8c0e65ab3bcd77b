"""Multi-FIB launches and the serving runtime on the GPU: every burst's next
hops equal the oracle's and its result alone; admission and eviction under a
tight memory budget; rebuild-and-swap of a live table."""
import numpy as np
import pytest

import planb_synth as S
from helpers import host_u16, say, to_dev
from oracle.trie import Trie

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    from paper_2604_14650_amd import planb
    return planb


@pytest.fixture(scope="module")
def vrfs():
    """Six VRF-style tables (tiny histogram + ::/0), 2k..60k prefixes."""
    sizes = [2000, 5000, 9000, 20000, 35000, 60000]
    tabs = [S.make_fib(S.vrf_spec(n), 9000 + k) for k, n in enumerate(sizes)]
    tries = [Trie(t.prefixes, t.lengths, t.next_hops) for t in tabs]
    return tabs, tries


def _bursts(tabs, count, seed, lo=1, hi=4096):
    rng = np.random.default_rng(seed)
    sizes = S.log_uniform_sizes(rng, count, lo, hi)
    tids = rng.integers(0, len(tabs), size=count)
    addrs = [S.mixed_traffic(tabs[t], int(n), 0.5, int(rng.integers(0, 2**62))) for t, n in zip(tids, sizes)]
    return sizes, tids, addrs


def test_multi_fib_launch(P, vrfs):
    import torch
    tabs, tries = vrfs
    ts = P.TableSet(8)
    fibs = [P.planb_build(t.prefixes, t.lengths, t.next_hops, fanout=16) for t in tabs]
    for k, f in enumerate(fibs):
        ts.set(k, f)
    sizes, tids, addrs = _bursts(tabs, 200, 1)
    sizes[3] = 0
    addrs[3] = addrs[3][:0]
    tids[5] = 7  # an empty slot: skipped
    flat = np.concatenate(addrs)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    d = to_dev(flat)
    out = torch.full((len(flat),), -1, dtype=torch.int16, device="cuda")
    rows = [(int(tids[i]), d[offs[i]:], out[offs[i]:], int(sizes[i])) if sizes[i] else (int(tids[i]), 0, 0, 0)
            for i in range(len(sizes))]
    desc = torch.from_numpy(np.frombuffer(bytes(P.burst_array(rows)), dtype=np.uint8).copy()).cuda()
    cnt = torch.tensor([len(rows)], dtype=torch.int32, device="cuda")
    for kpl in (1, 4, 16):
        ts.set_tuning(kpl, 2, 512)
        out.fill_(-1)
        P.planb_lookup_multi(ts, desc, cnt, len(rows))
        got = host_u16(out, len(flat))
        for i in range(len(sizes)):
            seg = got[offs[i]:offs[i + 1]]
            if tids[i] == 7:
                assert np.all(seg == 0xFFFF)
            elif sizes[i]:
                assert np.array_equal(seg, tries[tids[i]].lookup(addrs[i])), (kpl, i)


def test_multi_fib_learned_launch(P, vrfs):
    """Learned multi-FIB lookups equal the oracle burst by burst, tables with
    and without a trained model mixed in one launch (one slot empty)."""
    import torch
    tabs, tries = vrfs
    ts = P.TableSet(8)
    fibs = [P.planb_build(t.prefixes, t.lengths, t.next_hops, fanout=16) for t in tabs]
    for k, f in enumerate(fibs):
        if k % 2 == 0:
            P.planb_train(f, seed=k)
        ts.set(k, f)  # set after training: the slot takes the model as it is now
    sizes, tids, addrs = _bursts(tabs, 200, 6)
    sizes[4] = 0
    addrs[4] = addrs[4][:0]
    tids[7] = 7  # an empty slot: skipped
    flat = np.concatenate(addrs)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    d = to_dev(flat)
    out = torch.full((len(flat),), -1, dtype=torch.int16, device="cuda")
    rows = [(int(tids[i]), d[offs[i]:], out[offs[i]:], int(sizes[i])) if sizes[i] else (int(tids[i]), 0, 0, 0)
            for i in range(len(sizes))]
    desc = torch.from_numpy(np.frombuffer(bytes(P.burst_array(rows)), dtype=np.uint8).copy()).cuda()
    cnt = torch.tensor([len(rows)], dtype=torch.int32, device="cuda")
    fb = torch.zeros(1, dtype=torch.int32, device="cuda")
    P.planb_lookup_multi_learned(ts, desc, cnt, len(rows), fb)
    got = host_u16(out, len(flat))
    say(f"learned multi-FIB fallbacks {int(fb.item())} of {len(flat)}")
    for i in range(len(sizes)):
        seg = got[offs[i]:offs[i + 1]]
        if tids[i] == 7:
            assert np.all(seg == 0xFFFF)
        elif sizes[i]:
            assert np.array_equal(seg, tries[tids[i]].lookup(addrs[i])), i


def test_multi_fib_learned_long_runs(P, vrfs):
    """Enough bursts (3000, 32..4096 addresses) that each wavefront takes a
    run of many consecutive tiles, crossing bursts, tables with and without a
    model, and empty bursts: every burst equals the oracle."""
    import torch
    tabs, tries = vrfs
    ts = P.TableSet(len(tabs))
    fibs = [P.planb_build(t.prefixes, t.lengths, t.next_hops, fanout=16) for t in tabs]
    for k, f in enumerate(fibs):
        if k != 3:  # table 3 keeps no model: the tree descent inside the runs
            P.planb_train(f, seed=k, epochs=2)
        ts.set(k, f)
    sizes, tids, addrs = _bursts(tabs, 3000, 21, lo=32, hi=4096)
    for i in (5, 1500, 2999):
        sizes[i] = 0
        addrs[i] = addrs[i][:0]
    flat = np.concatenate(addrs)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    say(f"learned multi-FIB long runs: {len(sizes)} bursts, {len(flat)} lookups")
    d = to_dev(flat)
    out = torch.full((len(flat),), -1, dtype=torch.int16, device="cuda")
    rows = [(int(tids[i]), d[offs[i]:], out[offs[i]:], int(sizes[i])) if sizes[i] else (int(tids[i]), 0, 0, 0)
            for i in range(len(sizes))]
    desc = torch.from_numpy(np.frombuffer(bytes(P.burst_array(rows)), dtype=np.uint8).copy()).cuda()
    cnt = torch.tensor([len(rows)], dtype=torch.int32, device="cuda")
    P.planb_lookup_multi_learned(ts, desc, cnt, len(rows))
    got = host_u16(out, len(flat))
    for i in range(len(sizes)):
        if sizes[i]:
            assert np.array_equal(got[offs[i]:offs[i + 1]], tries[tids[i]].lookup(addrs[i])), i


def test_learned_server_equals_oracle(P, vrfs):
    tabs, tries = vrfs
    srv = P.Server(max_tables=len(tabs), streams=2, max_bursts=64, max_lookups=1 << 16, fanout=16, key_bits=64,
                   learned=True)
    for k, t in enumerate(tabs):
        srv.set_table(k, t.prefixes, t.lengths, t.next_hops)
    sizes, tids, addrs = _bursts(tabs, 200, 7)
    outs, done = _serve(P, srv, tabs, sizes, tids, addrs)
    st = srv.stats()
    say(f"learned server stats {st}")
    assert st["bursts"] == len(addrs) and st["admissions"] == len(tabs)
    for i in range(len(addrs)):
        assert np.array_equal(outs[i], tries[tids[i]].lookup(addrs[i])), i
    srv.close()


def _serve(P, srv, tabs, sizes, tids, addrs, poll_every=3):
    outs = [np.full(len(a), 0xFFFF, np.uint16) for a in addrs]
    done = {}
    for i in range(len(addrs)):
        srv.submit(int(tids[i]), addrs[i], outs[i], i)
        if i % poll_every == 0:
            for c in srv.poll():
                done[c[0]] = c
    while len(done) < len(addrs):
        for c in srv.poll(block=True):
            done[c[0]] = c
    return outs, done


@pytest.mark.parametrize("streams", [1, 3])
def test_server_mix_equals_alone_and_oracle(P, vrfs, streams):
    import torch
    tabs, tries = vrfs
    srv = P.Server(max_tables=len(tabs), streams=streams, max_bursts=64, max_lookups=1 << 16, fanout=16, key_bits=64)
    for k, t in enumerate(tabs):
        srv.set_table(k, t.prefixes, t.lengths, t.next_hops)
    sizes, tids, addrs = _bursts(tabs, 300, 2)
    outs, done = _serve(P, srv, tabs, sizes, tids, addrs)
    st = srv.stats()
    say(f"server streams={streams} stats {st}")
    assert st["bursts"] == len(addrs) and st["launches"] > 1
    alone_fibs = [P.planb_build(t.prefixes, t.lengths, t.next_hops, fanout=16) for t in tabs]
    for i in range(len(addrs)):
        assert np.array_equal(outs[i], tries[tids[i]].lookup(addrs[i])), i
        d = to_dev(addrs[i])
        o = torch.empty(len(addrs[i]), dtype=torch.int16, device="cuda")
        P.planb_lookup(alone_fibs[tids[i]], d, len(addrs[i]), o)
        assert np.array_equal(outs[i], host_u16(o, len(addrs[i]))), i
        assert done[i][4] >= done[i][3]
    srv.close()


def test_server_tight_budget_admission_and_eviction(P, vrfs):
    tabs, tries = vrfs
    probe = [P.planb_build(t.prefixes, t.lengths, t.next_hops, fanout=8) for t in tabs]
    total = sum(P.planb_get_info(f)["key_bytes"] + P.planb_get_info(f)["value_bytes"] for f in probe)
    del probe
    srv = P.Server(max_tables=len(tabs), streams=2, max_bursts=32, max_lookups=1 << 15, fanout=8, key_bits=64,
                   memory_budget=int(total * 0.6))
    for k, t in enumerate(tabs):
        srv.set_table(k, t.prefixes, t.lengths, t.next_hops)
    sizes, tids, addrs = _bursts(tabs, 240, 3, hi=2048)
    outs, _ = _serve(P, srv, tabs, sizes, tids, addrs, poll_every=1)
    st = srv.stats()
    say(f"tight budget stats {st} total={total}")
    assert st["evictions"] > 0 and st["admissions"] > len(tabs)
    assert st["resident_bytes"] <= int(total * 0.6)
    for i in range(len(addrs)):
        assert np.array_equal(outs[i], tries[tids[i]].lookup(addrs[i])), i
    srv.close()


def test_server_rejects_a_table_larger_than_the_budget(P, vrfs):
    """A burst whose table alone exceeds the budget completes with
    PLANB_ERANGE and an untouched output; bursts of a table that fits are
    served beside it, and the server keeps serving after the error."""
    tabs, tries = vrfs
    small = P.planb_build(tabs[0].prefixes, tabs[0].lengths, tabs[0].next_hops, fanout=16, key_bits=64)
    budget = P.planb_get_info(small)["key_bytes"] + P.planb_get_info(small)["value_bytes"] + 4096
    small.close()
    srv = P.Server(max_tables=2, streams=1, fanout=16, key_bits=64, memory_budget=budget)
    srv.set_table(0, tabs[-1].prefixes, tabs[-1].lengths, tabs[-1].next_hops)  # too large for the budget
    srv.set_table(1, tabs[0].prefixes, tabs[0].lengths, tabs[0].next_hops)
    big_out = np.full(10, 7, np.uint16)
    srv.submit(0, S.mixed_traffic(tabs[-1], 10, 0.5, 1), big_out, 0)
    a1 = S.mixed_traffic(tabs[0], 500, 0.5, 2)
    o1 = np.zeros(len(a1), np.uint16)
    srv.submit(1, a1, o1, 1)
    got = {}
    while len(got) < 2:
        for c in srv.poll(block=True):
            got[c[0]] = c
    assert got[0][5] == P.PLANB_ERANGE and (big_out == 7).all()
    assert got[1][5] == P.PLANB_OK and np.array_equal(o1, tries[0].lookup(a1))
    a2 = S.mixed_traffic(tabs[0], 300, 0.5, 3)  # polling again after the error
    o2 = np.zeros(len(a2), np.uint16)
    srv.submit(1, a2, o2, 2)
    c = srv.poll(block=True)
    assert [x[0] for x in c] == [2] and c[0][5] == P.PLANB_OK
    assert np.array_equal(o2, tries[0].lookup(a2))
    srv.close()


def test_server_rebuild_and_swap(P, vrfs):
    tabs, tries = vrfs
    old, new = tabs[1], tabs[2]
    t_old, t_new = tries[1], tries[2]
    srv = P.Server(max_tables=1, streams=2, max_bursts=16, max_lookups=1 << 14, fanout=16, key_bits=64)
    srv.set_table(0, old.prefixes, old.lengths, old.next_hops)
    a1 = S.mixed_traffic(old, 3000, 0.5, 11)
    o1 = np.zeros(len(a1), np.uint16)
    srv.submit(0, a1, o1, 1)
    srv.poll()  # launches burst 1 on the old table
    srv.set_table(0, new.prefixes, new.lengths, new.next_hops)  # swap while it may be in flight
    a2 = S.mixed_traffic(new, 3000, 0.5, 12)
    o2 = np.zeros(len(a2), np.uint16)
    srv.submit(0, a2, o2, 2)
    got = {}
    while len(got) < 2:
        for c in srv.poll(block=True):
            got[c[0]] = c
    assert np.array_equal(o1, t_old.lookup(a1))
    assert np.array_equal(o2, t_new.lookup(a2))
    srv.close()


def test_server_swap_while_launches_are_queued(P, vrfs):
    """A swap lands while launches of the old table are still enqueued
    behind a large copy and kernel on the other slot stream; every burst
    equals the oracle of the rules it was submitted under."""
    tabs, tries = vrfs
    old, new = tabs[5], tabs[0]  # the rebuilt rule set is small, so the swap itself is quick
    srv = P.Server(max_tables=1, streams=2, max_bursts=16, max_lookups=1 << 20, fanout=16, key_bits=64)
    srv.set_table(0, old.prefixes, old.lengths, old.next_hops)
    srv.admit(0)
    before = [S.mixed_traffic(old, 1 << 20, 0.5, 21), S.mixed_traffic(old, 2000, 0.5, 22)]
    outs = [np.zeros(len(a), np.uint16) for a in before]
    got = {}
    for k, a in enumerate(before):
        srv.submit(0, a, outs[k], k)
        for c in srv.poll():  # each poll fills a free slot: both launches are now enqueued
            got[c[0]] = c
    srv.set_table(0, new.prefixes, new.lengths, new.next_hops)
    after = S.mixed_traffic(new, 3000, 0.5, 23)
    o_after = np.zeros(len(after), np.uint16)
    srv.submit(0, after, o_after, 2)
    while len(got) < 3:
        for c in srv.poll(block=True):
            got[c[0]] = c
    assert all(c[5] == P.PLANB_OK for c in got.values())
    for k, a in enumerate(before):
        assert np.array_equal(outs[k], tries[5].lookup(a)), k
    assert np.array_equal(o_after, tries[0].lookup(after))
    srv.close()


def test_serving_replay_reports_latency(P, vrfs):
    from paper_2604_14650_amd import serve
    tabs, tries = vrfs
    srv = P.Server(max_tables=len(tabs), streams=2, max_bursts=256, max_lookups=1 << 18, fanout=16, key_bits=64)
    for k, t in enumerate(tabs):
        srv.set_table(k, t.prefixes, t.lengths, t.next_hops)
    sizes, tids, addrs = _bursts(tabs, 400, 4, lo=32)
    arrivals = np.cumsum(np.random.default_rng(5).exponential(1e-5, size=len(sizes)))
    outs = [np.zeros(len(a), np.uint16) for a in addrs]
    lat, wall = serve.replay(srv, arrivals, tids, addrs, outs)
    s = serve.summary(lat, sizes, wall)
    say(f"replay summary {s}")
    assert s["p99_us"] >= s["p50_us"] > 0
    for i in range(len(addrs)):
        assert np.array_equal(outs[i], tries[tids[i]].lookup(addrs[i]))
    # the native replay, tables admitted beforehand
    for k in range(len(tabs)):
        srv.admit(k)
    lat, wall, outs = serve.replay_native(srv, arrivals, tids, addrs)
    s = serve.summary(lat, sizes, wall)
    say(f"native replay summary {s}")
    assert s["p99_us"] >= s["p50_us"] > 0
    for i in range(len(addrs)):
        assert np.array_equal(outs[i], tries[tids[i]].lookup(addrs[i]))
    srv.close()


@pytest.mark.parametrize("learned", [False, True])
def test_zero_copy_server_equals_oracle(P, vrfs, learned):
    """Zero-copy serving: the kernels read the bursts from, and write the next
    hops to, registered pinned host memory; every burst equals the oracle, and
    a burst outside the registered memory is refused before any launch."""
    from paper_2604_14650_amd import serve
    tabs, tries = vrfs
    srv = P.Server(max_tables=len(tabs), streams=3, max_bursts=64, max_lookups=1 << 16, fanout=16, key_bits=64,
                   learned=learned, zero_copy=True)
    for k, t in enumerate(tabs):
        srv.set_table(k, t.prefixes, t.lengths, t.next_hops)
    sizes, tids, addrs = _bursts(tabs, 300, 11)
    io = serve.pinned_io(addrs)
    say(f"zero-copy server learned={learned}: {int(sizes.sum())} lookups in {len(addrs)} bursts")
    lat, wall, outs = serve.replay_zero_copy(srv, np.zeros(len(addrs)), tids, io)
    for i in range(len(addrs)):
        assert np.array_equal(outs[i], tries[tids[i]].lookup(addrs[i])), i
    # arrivals spread out: the same results
    lat, wall, outs2 = serve.replay_zero_copy(srv, np.arange(len(addrs)) * 2e-6, tids, io)
    assert all(np.array_equal(a, b) for a, b in zip(outs, outs2))
    pageable = np.zeros((16, 2), np.uint64)
    with pytest.raises(P.PlanbError) as e:
        srv.submit(0, pageable, np.zeros(16, np.uint16), 99)
    assert e.value.code == P.PLANB_EINVAL
    srv.close()


def test_zero_copy_registration_refuses_pageable_memory(P, vrfs):
    tabs, _ = vrfs
    srv = P.Server(max_tables=2, streams=1, max_bursts=16, max_lookups=1 << 12, fanout=16, key_bits=64,
                   zero_copy=True)
    buf = np.zeros(4096, np.uint64)
    with pytest.raises(P.PlanbError) as e:
        srv.register_io(buf.ctypes.data, buf.nbytes)
    assert e.value.code == P.PLANB_EINVAL
    srv.close()
