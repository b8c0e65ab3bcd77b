"""A FIB freed while lookups on it are still running on another stream
(Section 3.6: the replaced structure is freed once the lookups in flight on
it complete): planb_free returns before that stream finishes, the memory is
released only after it, and the lookups' results equal the oracle's even
when new FIBs are built and searched right after the free."""
import numpy as np
import pytest

import planb_synth as S
from helpers import fib_of, host_u16, oracle_trie, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    from paper_2604_14650_amd import planb
    return planb


def test_free_while_another_stream_looks_up(P):
    import torch
    fib = fib_of("backbone", 22)
    n, reps = 1 << 23, 8
    addrs = S.backbone_traffic(fib, n, seed=4022)
    want = oracle_trie("backbone", 22).lookup(addrs)
    d = to_dev(addrs)
    outs = [torch.full((n,), -1, dtype=torch.int16, device="cuda") for _ in range(reps)]
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, fanout=8)
    torch.cuda.synchronize()
    s1 = torch.cuda.Stream()
    say(f"free while {reps} lookups of {n} run on a side stream")
    for o in outs:
        P.planb_lookup(h, d, n, o, stream=s1)
    h.close()  # planb_free: must neither wait for s1 nor free under it
    still_running = not s1.query()
    # new structures of the same size, built and searched at once, reuse freed memory
    # only after s1's lookups are done
    other = fib_of("backbone", 23)
    h2 = P.planb_build(other.prefixes, other.lengths, other.next_hops, fanout=8)
    o2 = torch.empty(n, dtype=torch.int16, device="cuda")
    P.planb_lookup(h2, d, n, o2)
    s1.synchronize()
    torch.cuda.synchronize()
    for k, o in enumerate(outs):
        assert np.array_equal(host_u16(o, n), want), k
    assert np.array_equal(host_u16(o2, n), oracle_trie("backbone", 23).lookup(addrs))
    assert still_running, "planb_free waited for the other stream's lookups"
    h2.close()


def test_free_of_a_trained_fib_while_learned_lookups_run(P):
    import torch
    fib = fib_of("tiny", 11)
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops)
    P.planb_train(h, seed=3)
    n = 1 << 20
    addrs = S.tiny_traffic(fib, n, seed=77)
    want = oracle_trie("tiny", 11).lookup(addrs)
    d = to_dev(addrs)
    s1 = torch.cuda.Stream()
    outs = [torch.full((n,), -1, dtype=torch.int16, device="cuda") for _ in range(4)]
    for o in outs:
        P.planb_lookup_learned(h, d, n, o, stream=s1)
    h.close()
    h2 = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops)
    P.planb_train(h2, seed=4)  # new model memory while the old lookups may still run
    s1.synchronize()
    for o in outs:
        assert np.array_equal(host_u16(o, n), want)
    h2.close()


def test_table_set_slot_change_waits_for_enqueued_launches(P):
    import torch
    tabs = [fib_of("tiny", 11), S.make_fib(S.vrf_spec(20000), 9100)]
    fibs = [P.planb_build(t.prefixes, t.lengths, t.next_hops, fanout=16) for t in tabs]
    ts = P.TableSet(2)
    ts.set(0, fibs[0])
    n = 1 << 20
    addrs = S.tiny_traffic(tabs[0], n, seed=5)
    d = to_dev(addrs)
    out = torch.full((n,), -1, dtype=torch.int16, device="cuda")
    rows = [(0, d, out, n)]
    desc = torch.from_numpy(np.frombuffer(bytes(P.burst_array(rows)), dtype=np.uint8).copy()).cuda()
    cnt = torch.tensor([1], dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    s1 = torch.cuda.Stream()
    for _ in range(3):
        P.planb_lookup_multi(ts, desc, cnt, 1, stream=s1)
    ts.set(0, fibs[1])  # the enqueued launches must still read table 0 as it was
    s1.synchronize()
    assert np.array_equal(host_u16(out, n), oracle_trie("tiny", 11).lookup(addrs))
    ts.close()
