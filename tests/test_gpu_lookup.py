"""GPU parity of the plain lookup (build + planb_lookup through the C ABI)
against the CPU oracle: next hops must be identical, address for address."""
import numpy as np
import pytest

import planb_synth as S
from helpers import fib_of, host_u16, oracle_trie, out_u16, say, to_dev
from oracle.brute import lpm_bruteforce
from oracle.trie import lpm_trie

pytestmark = pytest.mark.gpu

M128 = (1 << 128) - 1

VARIANTS = [(8, 1, 1), (8, 2, 2), (8, 4, 4), (8, 8, 1), (16, 1, 2), (16, 2, 1), (16, 4, 2), (16, 4, 4),
            (16, 8, 2), (16, 16, 1), (32, 1, 1), (32, 2, 2), (32, 4, 2), (32, 8, 4), (32, 16, 1)]
# (fanout, keys_per_lane, R) with binary search in the LDS levels; keys_per_lane < fanout = hybrid
BIN_VARIANTS = [(8, 8, 1), (8, 8, 2), (8, 4, 4), (8, 2, 2), (16, 16, 1), (16, 8, 2), (16, 4, 4),
                (32, 32 // 2, 2), (32, 8, 1)]


def gpu_lookup(P, fib, addrs, fanout=16, kpl=None, lds=-1, R=2, key_bits=0, block=512):
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, fanout=fanout, key_bits=key_bits)
    if kpl is not None:
        P.planb_set_tuning(h, kpl, lds, R, block)
    d = to_dev(addrs)
    out = out_u16(addrs.shape[0])
    P.planb_lookup(h, d, addrs.shape[0], out)
    return host_u16(out, addrs.shape[0]), h


@pytest.fixture(scope="module")
def P():
    from paper_2604_14650_amd import planb
    return planb


@pytest.fixture(scope="module")
def tiny():
    fib = fib_of("tiny", 11)
    addrs = S.tiny_traffic(fib, 1 << 20, seed=1011)
    return fib, addrs, oracle_trie("tiny", 11).lookup(addrs)


@pytest.mark.parametrize("key_bits", [0, 128])
@pytest.mark.parametrize("fanout,kpl,R", VARIANTS)
def test_tiny_all_addresses(P, tiny, fanout, kpl, R, key_bits):
    fib, addrs, want = tiny
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, fanout=fanout, key_bits=key_bits)
    info = P.planb_get_info(h)
    assert info["key_bits"] == (key_bits or 64)  # every tiny prefix is at most /64
    depth = info["depth"]
    d = to_dev(addrs)
    for lds, block in sorted({(0, 512), (-1, 512), (depth, 1024), (max(0, depth - 1), 512)}):
        say(f"tiny key_bits={key_bits} fanout={fanout} kpl={kpl} R={R} lds={lds} block={block}")
        try:
            P.planb_set_tuning(h, kpl, lds, R, block)
        except P.PlanbError:
            continue  # more levels than fit in LDS
        out = out_u16(addrs.shape[0])
        P.planb_lookup(h, d, addrs.shape[0], out)
        got = host_u16(out, addrs.shape[0])
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, f"{bad.size} mismatches, first at {bad[:5]}"


@pytest.mark.parametrize("key_bits", [0, 128])
@pytest.mark.parametrize("fanout,kpl,R", BIN_VARIANTS)
def test_tiny_binary_search_in_lds(P, tiny, fanout, kpl, R, key_bits):
    fib, addrs, want = tiny
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, fanout=fanout, key_bits=key_bits)
    depth = P.planb_get_info(h)["depth"]
    d = to_dev(addrs)
    for lds in sorted({0, 1, depth - 1, depth}):
        say(f"tiny binary key_bits={key_bits} fanout={fanout} kpl={kpl} R={R} lds={lds}")
        P.planb_set_tuning(h, kpl, lds, R, 1024, 1)
        out = out_u16(addrs.shape[0])
        P.planb_lookup(h, d, addrs.shape[0], out)
        assert np.array_equal(host_u16(out, addrs.shape[0]), want)


def _edge_fibs():
    base = 0x20010DB8 << 96
    return {
        "empty": [],
        "default_only": [(0, 0, 42)],
        "top_of_space": [(0, 0, 1), (0xFFFF << 112, 16, 2), (M128, 128, 3), (M128 - 1, 128, 4)],
        "nested_shared_start": [(base, 32, 1), (base, 48, 2), (base, 64, 3), (base | (5 << 60), 68, 4),
                                (base | (5 << 60) | 77, 128, 5)],
        "zero_host_route": [(0, 128, 7), (1, 128, 8), (0, 1, 9)],
    }


def _edge_queries(rules, rng):
    q = {0, 1, M128, M128 - 1, 1 << 127, (1 << 127) - 1}
    for Pv, Lv, _ in rules:
        end = Pv + (1 << (128 - Lv)) - 1
        for v in (Pv - 1, Pv, Pv + 1, end - 1, end, end + 1):
            if 0 <= v <= M128:
                q.add(v)
    q |= {int(x) << 64 | int(y) for x, y in rng.integers(0, 2**63, size=(300, 2))}
    return S.from_ints(sorted(q))


@pytest.mark.parametrize("fanout", [8, 16, 32])
@pytest.mark.parametrize("name", sorted(_edge_fibs()))
def test_edge_cases(P, fanout, name):
    rules = _edge_fibs()[name]
    rng = np.random.default_rng(7)
    p = S.from_ints([r[0] for r in rules]) if rules else np.zeros((0, 2), np.uint64)
    L = np.array([r[1] for r in rules], np.uint8)
    nh = np.array([r[2] for r in rules], np.uint16)
    q = _edge_queries(rules, rng)
    want = lpm_bruteforce(p, L, nh, q)
    fib = S.Fib(p, L, nh)
    for kpl in (1, fanout // 2, fanout // 4):
        if fanout // kpl > 32:
            continue
        for key_bits in (0, 128):
            say(f"edge {name} fanout={fanout} kpl={kpl} key_bits={key_bits}")
            got, _ = gpu_lookup(P, fib, q, fanout, kpl, -1, 2, key_bits)
            assert np.array_equal(got, want)
            got, _ = gpu_lookup(P, fib, q, fanout, kpl, 0, 1, key_bits, 1024)
            assert np.array_equal(got, want)
    for key_bits in (0, 128):  # binary search in the LDS levels (whole tree, or with hybrid lower levels)
        h = P.planb_build(p, L, nh, fanout=fanout, key_bits=key_bits)
        depth = P.planb_get_info(h)["depth"]
        d = to_dev(q)
        for kpl, lds in ((fanout, depth), (fanout // 2, depth - 1), (fanout // 4, 0)):
            P.planb_set_tuning(h, kpl, lds, 2, 512, 1)
            out = out_u16(q.shape[0])
            P.planb_lookup(h, d, q.shape[0], out)
            assert np.array_equal(host_u16(out, q.shape[0]), want), (kpl, lds)


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 1000, 4097, 123457])
def test_ragged_batch_sizes(P, tiny, n):
    fib, addrs, want = tiny
    say(f"ragged n={n}")
    got, _ = gpu_lookup(P, fib, addrs[:n])
    assert np.array_equal(got, want[:n])


def test_zero_length_batch_is_a_noop(P, tiny):
    import torch
    fib, addrs, _ = tiny
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops)
    out = out_u16(4)
    P.planb_lookup(h, to_dev(addrs[:4]), 0, out)
    torch.cuda.synchronize()
    assert (out.cpu().numpy() == -1).all()


def test_misaligned_and_null_pointers_rejected(P, tiny):
    import torch
    fib, addrs, _ = tiny
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops)
    d = to_dev(addrs[:64])
    out = out_u16(64)
    with pytest.raises(P.PlanbError) as e:
        P.planb_lookup(h, d.data_ptr() + 8, 8, out)
    assert e.value.code == P.PLANB_EINVAL
    with pytest.raises(P.PlanbError):
        P.planb_lookup(h, 0, 8, out)
    with pytest.raises(P.PlanbError):
        P.planb_lookup(h, d, 8, out.data_ptr() + 1)
    torch.cuda.synchronize()


def test_interval_index_output_is_consistent(P, tiny):
    import torch
    fib, addrs, want = tiny
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops)
    starts, nh = P.planb_export_intervals(h)
    n = 1 << 16
    idx = torch.empty(n, dtype=torch.int32, device="cuda")
    P.planb_lookup_index(h, to_dev(addrs[:n]), n, idx)
    i = idx.cpu().numpy().astype(np.int64)
    assert i.min() >= 0 and i.max() < len(starts)
    assert np.array_equal(nh[i], want[:n])
    # the returned interval holds the address: starts[i] <= x < starts[i + 1]
    a = addrs[:n]
    s_hi, s_lo = starts[i, 0], starts[i, 1]
    assert np.all((s_hi < a[:, 0]) | ((s_hi == a[:, 0]) & (s_lo <= a[:, 1])))
    nx = np.minimum(i + 1, len(starts) - 1)
    last = i == len(starts) - 1
    n_hi, n_lo = starts[nx, 0], starts[nx, 1]
    assert np.all(last | (a[:, 0] < n_hi) | ((a[:, 0] == n_hi) & (a[:, 1] < n_lo)))


def test_two_streams_overlapping(P, tiny):
    import torch
    fib, addrs, want = tiny
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops)
    half = addrs.shape[0] // 2
    d = to_dev(addrs)
    out = out_u16(addrs.shape[0])
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    for _ in range(3):
        P.planb_lookup(h, d[:half], half, out[:half], stream=s1)
        P.planb_lookup(h, d[half:], addrs.shape[0] - half, out[half:], stream=s2)
    torch.cuda.synchronize()
    assert np.array_equal(host_u16(out, addrs.shape[0]), want)


@pytest.mark.parametrize("key_bits", [0, 128])
@pytest.mark.parametrize("fanout", [8, 16, 32])
def test_backbone_4m_addresses(P, fanout, key_bits):
    fib = fib_of("backbone", 22)
    addrs = S.backbone_traffic(fib, 1 << 22, seed=2022)
    want = oracle_trie("backbone", 22).lookup(addrs)
    say(f"backbone fanout={fanout} key_bits={key_bits}")
    got, _ = gpu_lookup(P, fib, addrs, fanout, key_bits=key_bits)
    assert np.array_equal(got, want)


def test_narrow_keys_refused_when_inexact(P):
    fib = fib_of("large", 33)  # holds /128 host routes
    with pytest.raises(P.PlanbError) as e:
        P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, key_bits=64)
    assert e.value.code == P.PLANB_EINVAL
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops)
    assert P.planb_get_info(h)["key_bits"] == 128


def test_large_fib_with_host_routes(P):
    fib = fib_of("large", 33)
    addrs = S.zipf_traffic(fib, 1 << 22, seed=3033)
    want = oracle_trie("large", 33).lookup(addrs)
    for fanout in (8, 16, 32):
        say(f"large fanout={fanout}")
        got, _ = gpu_lookup(P, fib, addrs, fanout)
        assert np.array_equal(got, want)


def test_brute_force_agrees_on_a_sample(P, tiny):
    fib, addrs, want = tiny
    got, _ = gpu_lookup(P, fib, addrs[:3000])
    assert np.array_equal(got, lpm_bruteforce(fib.prefixes, fib.lengths, fib.next_hops, addrs[:3000]))


@pytest.mark.parametrize("fanout", [8, 16, 32])
@pytest.mark.parametrize("name", sorted(_edge_fibs()))
def test_bsearch_baseline_edge_cases(P, fanout, name):
    """The sorted-array binary search baseline gives the oracle's answers."""
    rules = _edge_fibs()[name]
    rng = np.random.default_rng(9)
    p = S.from_ints([r[0] for r in rules]) if rules else np.zeros((0, 2), np.uint64)
    L = np.array([r[1] for r in rules], np.uint8)
    nh = np.array([r[2] for r in rules], np.uint16)
    q = _edge_queries(rules, rng)
    want = lpm_bruteforce(p, L, nh, q)
    for key_bits in (0, 128):
        say(f"bsearch edge {name} fanout={fanout} key_bits={key_bits}")
        h = P.planb_build(p, L, nh, fanout=fanout, key_bits=key_bits)
        out = out_u16(q.shape[0])
        P.planb_lookup_bsearch(h, to_dev(q), q.shape[0], out)
        assert np.array_equal(host_u16(out, q.shape[0]), want)


@pytest.mark.parametrize("key_bits", [0, 128])
def test_bsearch_baseline_tiny_and_backbone(P, tiny, key_bits):
    fib, addrs, want = tiny
    for fanout in (8, 16, 32):
        h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, fanout=fanout, key_bits=key_bits)
        out = out_u16(addrs.shape[0])
        P.planb_lookup_bsearch(h, to_dev(addrs), addrs.shape[0], out)
        assert np.array_equal(host_u16(out, addrs.shape[0]), want), fanout
    bb = fib_of("backbone", 22)
    a = S.backbone_traffic(bb, 1 << 21, seed=2023)
    h = P.planb_build(bb.prefixes, bb.lengths, bb.next_hops, fanout=8, key_bits=key_bits)
    out = out_u16(a.shape[0])
    P.planb_lookup_bsearch(h, to_dev(a), a.shape[0], out)
    assert np.array_equal(host_u16(out, a.shape[0]), oracle_trie("backbone", 22).lookup(a))


@pytest.mark.parametrize("with_top_rule", [False, True])
def test_top_of_space_narrow_keys(P, with_top_rule):
    """64-bit key slots: an address whose high word is all ones counts the
    sentinel padding of the last leaf too.  With a rule starting at
    ffff:ffff:ffff:ffff:: a real key equals the sentinel as well.  Both the
    next hop and the interval index must still be those of the last interval
    at or below the address."""
    import torch
    H = (1 << 64) - 1
    rules = [(0, 0, 1), (0xFFFF << 112, 16, 2), (0x2001 << 112, 16, 5), ((H - 1) << 64, 64, 4)]
    if with_top_rule:
        rules.append((H << 64, 64, 3))
    p = S.from_ints([r[0] for r in rules])
    L = np.array([r[1] for r in rules], np.uint8)
    nh = np.array([r[2] for r in rules], np.uint16)
    rng = np.random.default_rng(21)
    his = [H, H - 1, H - 2, 0xFFFF << 48, (0xFFFF << 48) - 1, 0x2001 << 48, 0]
    los = [0, 1, H, H - 1] + [int(v) for v in rng.integers(0, 2**63, size=4)]
    q = S.from_ints(sorted({h << 64 | lo for h in his for lo in los}))
    want = lpm_bruteforce(p, L, nh, q)
    for fanout, kpl in ((8, 2), (16, 4), (32, 8), (8, 1), (16, 16)):
        h = P.planb_build(p, L, nh, fanout=fanout)
        assert P.planb_get_info(h)["key_bits"] == 64
        starts, ivnh = P.planb_export_intervals(h)
        depth = P.planb_get_info(h)["depth"]
        for lds, R, bin_ in ((0, 2, 0), (-1, 1, 0), (max(0, depth - 1), 2, 1), (depth, 2, 1)):
            say(f"top of space narrow fanout={fanout} kpl={kpl} lds={lds} R={R} bin={bin_} top={with_top_rule}")
            try:
                P.planb_set_tuning(h, kpl, lds, R, 512, bin_)
            except P.PlanbError:
                continue  # binary search needs fanout / keys_per_lane in {1, 2, 4}
            out = out_u16(q.shape[0])
            P.planb_lookup(h, to_dev(q), q.shape[0], out)
            assert np.array_equal(host_u16(out, q.shape[0]), want)
            idx = torch.full((q.shape[0],), -1, dtype=torch.int32, device="cuda")
            P.planb_lookup_index(h, to_dev(q), q.shape[0], idx)
            i = idx.cpu().numpy().astype(np.int64)
            assert np.array_equal(ivnh[i], want)
            # the interval is the last one whose start (high word) is <= the address's
            assert np.array_equal(i, np.searchsorted(starts[:, 0], q[:, 0], side="right") - 1)


TOPS_SHAPES = [(8, 2, 1), (8, 2, 2), (8, 4, 2), (8, 4, 4), (16, 4, 2), (16, 8, 1), (32, 8, 2), (32, 16, 4)]


@pytest.mark.parametrize("key_bits", [0, 128])
@pytest.mark.parametrize("fanout,kpl,R", TOPS_SHAPES)
def test_key_tops_in_lds_tiny(P, tiny, fanout, kpl, R, key_bits):
    """lds_search 2: every internal level in LDS, the bottom one as 32-bit key
    tops, exact on ties, with 64- and with 128-bit key slots; next hops and
    interval indices equal the oracle's."""
    import torch
    fib, addrs, want = tiny
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, fanout=fanout, key_bits=key_bits)
    starts, ivnh = P.planb_export_intervals(h)
    d = to_dev(addrs)
    for block in (512, 1024):
        say(f"tops tiny fanout={fanout} kpl={kpl} R={R} block={block} key_bits={key_bits}")
        P.planb_set_tuning(h, kpl, -1, R, block, 2)
        assert P.planb_get_tuning(h)["lds_search"] == 2
        out = out_u16(addrs.shape[0])
        P.planb_lookup(h, d, addrs.shape[0], out)
        assert np.array_equal(host_u16(out, addrs.shape[0]), want)
    # 3 fewer addresses: below 2^20 the same tuning runs the whole-key hybrid descent
    m = addrs.shape[0] - 3
    out = out_u16(m)
    P.planb_lookup(h, d, m, out)
    assert np.array_equal(host_u16(out, m), want[:m])
    n = addrs.shape[0]
    idx = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    P.planb_lookup_index(h, d, n, idx)
    i = idx.cpu().numpy().astype(np.int64)
    assert np.array_equal(i, np.searchsorted(starts[:, 0], addrs[:, 0], side="right") - 1)


@pytest.mark.parametrize("fanout,key_bits", [(8, 0), (16, 0), (16, 128)])
def test_key_tops_in_lds_backbone(P, fanout, key_bits):
    """The backbone-shaped table: its addresses inside /48 prefixes often tie
    a boundary's top 32 bits, so the exact re-read is exercised heavily."""
    fib = fib_of("backbone", 22)
    a = S.backbone_traffic(fib, 1 << 21, seed=77)
    want = oracle_trie("backbone", 22).lookup(a)
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, fanout=fanout, key_bits=key_bits)
    for kpl, R, block in ((fanout // 4, 2, 1024), (fanout // 2, 1, 512)):
        say(f"tops backbone fanout={fanout} key_bits={key_bits} kpl={kpl} R={R} block={block}")
        try:
            P.planb_set_tuning(h, kpl, -1, R, block, 2)
        except P.PlanbError as e:
            assert e.code == P.PLANB_ERANGE  # the tops exceed a workgroup's LDS
            continue
        out = out_u16(a.shape[0])
        P.planb_lookup(h, to_dev(a), a.shape[0], out)
        assert np.array_equal(host_u16(out, a.shape[0]), want)


@pytest.mark.parametrize("name", ["empty", "default_only", "nested_shared_start_64", "top_64"])
def test_key_tops_in_lds_edges(P, name):
    H = (1 << 64) - 1
    base = 0x20010DB8 << 96
    rules = {
        "empty": [],
        "default_only": [(0, 0, 42)],
        "nested_shared_start_64": [(base, 32, 1), (base, 48, 2), (base, 64, 3), (base | (5 << 70), 60, 4),
                                   (base | (1 << 64), 64, 5), (base | (2 << 64), 63, 6)],
        "top_64": [(0, 0, 1), (0xFFFF << 112, 16, 2), ((H - 1) << 64, 64, 4), (H << 64, 64, 3),
                   ((H - 7) << 64, 61, 9)],
    }[name]
    p = S.from_ints([r[0] for r in rules]) if rules else np.zeros((0, 2), np.uint64)
    L = np.array([r[1] for r in rules], np.uint8)
    nh = np.array([r[2] for r in rules], np.uint16)
    rng = np.random.default_rng(5)
    q = _edge_queries(rules, rng)
    # addresses sharing the top 32 bits of every boundary, above and below it
    extra = set()
    for Pv, Lv, _ in rules:
        for v in (Pv, Pv + (1 << (128 - Lv))):
            hi = (v >> 64) & H
            for d in (-(1 << 40), -1, 0, 1, 1 << 31):
                h2 = hi + d
                if 0 <= h2 <= H and (h2 >> 32) == (hi >> 32):
                    extra.add(h2 << 64 | int(rng.integers(0, 2**63)))
    q = S.from_ints(sorted({S.to_int(r) for r in q} | extra)) if extra else q
    want = lpm_bruteforce(p, L, nh, q)
    # repeated to 2^20 addresses: smaller batches run the whole-key hybrid descent
    reps = -(-(1 << 20) // q.shape[0])
    q, want = np.tile(q, (reps, 1)), np.tile(want, reps)
    for fanout in (8, 16, 32):
        h = P.planb_build(p, L, nh, fanout=fanout, key_bits=64)  # automatic would pick 32 for the first two
        for kpl, R in ((fanout // 2, 2), (fanout // 4, 1)):
            say(f"tops edge {name} fanout={fanout} kpl={kpl} R={R}")
            P.planb_set_tuning(h, kpl, -1, R, 1024, 2)
            out = out_u16(q.shape[0])
            P.planb_lookup(h, to_dev(q), q.shape[0], out)
            assert np.array_equal(host_u16(out, q.shape[0]), want)


@pytest.mark.parametrize("background", [190, 201, 213])
def test_key_tops_ties_at_the_top_of_the_space(P, background):
    """lds_search 2 on trees whose last leaves start with keys whose top 32 bits
    are all ones: an address with that top ties those separators and the
    sentinel slots after the last leaf, and walks back over several leaves
    (each tie read comes from a leaf's first slot, clamped to the last leaf).
    Fill levels vary with the background, so the last bottom node ends at
    different slots."""
    from oracle.brute import lpm_bruteforce_np
    H = (1 << 64) - 1
    TOP = 0xFFFFFFFF << 32
    rng = np.random.default_rng(background)
    rules = [(0, 0, 1)]
    for k, v in enumerate(rng.choice(1 << 16, size=background, replace=False)):
        hi = (0x20010DB8 << 32) | (int(v) << 16)
        rules.append((hi << 64, 48, 2 + k % 1000))
    tops_hi = sorted({TOP | int(v) for v in rng.integers(0, 1 << 32, size=15)})
    for k, hi in enumerate(tops_hi):
        rules.append((hi << 64, 64, 3000 + k))
    p = S.from_ints([r[0] for r in rules])
    L = np.array([r[1] for r in rules], np.uint8)
    nh = np.array([r[2] for r in rules], np.uint16)
    his = {H, H - 1, TOP, TOP - 1, TOP + 1}
    for hi in tops_hi:
        his |= {hi - 1, hi, hi + 1, hi + 2}
    his |= {TOP | int(v) for v in rng.integers(0, 1 << 32, size=200)}
    his |= {(0x20010DB8 << 32) | int(v) for v in rng.integers(0, 1 << 32, size=200)}
    q = S.from_ints(sorted(h << 64 | int(rng.integers(0, 2**63)) for h in his))
    want = lpm_bruteforce_np(p, L, nh, q)
    reps = -(-(1 << 20) // q.shape[0])  # at least 2^20 lookups: the key-tops kernel runs
    q, want = np.tile(q, (reps, 1)), np.tile(want, reps)
    d = to_dev(q)
    for fanout in (8, 16, 32):
        h = P.planb_build(p, L, nh, fanout=fanout, key_bits=64)
        assert P.planb_get_info(h)["depth"] >= 2
        for kpl, R in ((fanout // 2, 2), (fanout // 4, 1)):
            say(f"tops top-of-space background={background} fanout={fanout} kpl={kpl} R={R}")
            P.planb_set_tuning(h, kpl, -1, R, 1024, 2)
            out = out_u16(q.shape[0])
            P.planb_lookup(h, d, q.shape[0], out)
            assert np.array_equal(host_u16(out, q.shape[0]), want)


def test_key_tops_refused_for_32bit_keys(P, tiny):
    fib, _, _ = tiny
    v4 = S.make_fib(S.IPV4_TINY, 40)
    h = P.planb_build(v4.prefixes, v4.lengths, v4.next_hops, fanout=8)
    assert P.planb_get_info(h)["key_bits"] == 32
    with pytest.raises(P.PlanbError) as e:
        P.planb_set_tuning(h, 2, -1, 2, 1024, 2)
    assert e.value.code == P.PLANB_EINVAL
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, fanout=8)
    with pytest.raises(P.PlanbError) as e:  # one lane per lookup in every level: no such shape
        P.planb_set_tuning(h, 8, -1, 2, 1024, 2)
    assert e.value.code == P.PLANB_EINVAL


def test_key_tops_dense_slash32(P):
    """20,000 /64 rules and 300 /48 rules inside one /32: hundreds of
    consecutive bottom-level keys share their top 32 bits, so the tie walk of
    lds_search 2 runs over long runs of equal tops."""
    rng = np.random.default_rng(41)
    top = 0x20010DB8 << 96
    los = rng.choice(1 << 32, size=20000, replace=False).astype(np.int64)
    rules = {(top | (int(v) << 64), 64): int(rng.integers(0, 60000)) for v in los}
    for v in rng.choice(1 << 16, size=300, replace=False):
        rules[(top | (int(v) << 80), 48)] = int(rng.integers(0, 60000))
    rules[(top, 32)] = 7
    rules[(0, 0)] = 1
    keys = sorted(rules)
    p = S.from_ints([k[0] for k in keys])
    L = np.array([k[1] for k in keys], np.uint8)
    nh = np.array([rules[k] for k in keys], np.uint16)
    from oracle.trie import Trie
    trie = Trie(p, L, nh)
    hi = np.concatenate([(top >> 64) + rng.integers(0, 1 << 32, size=(1 << 20) - 4096),
                         (p[rng.integers(0, len(keys), size=4096), 0]).astype(np.int64)]).astype(np.uint64)
    q = np.stack([hi, rng.integers(0, 2**63, size=hi.shape[0]).astype(np.uint64)], axis=1)
    want = trie.lookup(q)
    h = P.planb_build(p, L, nh, fanout=8)
    assert P.planb_get_info(h)["key_bits"] == 64
    say("tops dense /32")
    P.planb_set_tuning(h, 2, -1, 2, 1024, 2)
    out = out_u16(q.shape[0])
    P.planb_lookup(h, to_dev(q), q.shape[0], out)
    assert np.array_equal(host_u16(out, q.shape[0]), want)


def test_key_tops_refused_when_too_large(P):
    """A 300k-prefix table with 64-bit keys: its bottom internal level's tops
    exceed a workgroup's LDS, so lds_search 2 is refused with PLANB_ERANGE,
    the default tuning falls back to lds_search 1, and lookups stay exact."""
    from oracle.trie import Trie
    fib = S.make_fib(S.vrf_spec(300000), 91)
    h = P.planb_build(fib.prefixes, fib.lengths, fib.next_hops, fanout=8)
    assert P.planb_get_info(h)["key_bits"] == 64
    assert P.planb_get_tuning(h)["lds_search"] == 1
    with pytest.raises(P.PlanbError) as e:
        P.planb_set_tuning(h, 2, -1, 2, 1024, 2)
    assert e.value.code == P.PLANB_ERANGE
    a = S.mixed_traffic(fib, 1 << 20, 0.5, 123)
    say("tops refused: default tuning on a 300k table")
    out = out_u16(a.shape[0])
    P.planb_lookup(h, to_dev(a), a.shape[0], out)
    assert np.array_equal(host_u16(out, a.shape[0]), Trie(fib.prefixes, fib.lengths, fib.next_hops).lookup(a))


@pytest.mark.parametrize("fanout", [8, 16, 32])
def test_key_tops_wide_keys_tie_on_the_high_word(P, fanout):
    """128-bit key slots with the bottom level as key tops: /128 host routes,
    /96 and /112 rules and /64s that share their high word (and so their top
    32 bits) with many boundaries, queried on every boundary and one either
    side of it, so that ties are settled by comparing whole 128-bit keys."""
    rng = np.random.default_rng(17)
    rules = {(0, 0): 1}
    for k in range(300):
        hi = (0x20010DB8 << 32) | int(rng.integers(0, 1 << 20))
        rules[(hi << 64, 64)] = int(rng.integers(0, 60000))
        for _ in range(8):
            lo = int(rng.integers(0, 1 << 63))
            ln = int(rng.choice([96, 112, 120, 128]))
            pfx = (hi << 64 | lo) >> (128 - ln) << (128 - ln)
            rules[(pfx, ln)] = int(rng.integers(0, 60000))
    keys = sorted(rules)
    p = S.from_ints([k[0] for k in keys])
    L = np.array([k[1] for k in keys], np.uint8)
    nh = np.array([rules[k] for k in keys], np.uint16)
    h = P.planb_build(p, L, nh, fanout=fanout)
    assert P.planb_get_info(h)["key_bits"] == 128
    starts, _ = P.planb_export_intervals(h)
    pts = set()
    for hi, lo in starts:
        v = int(hi) << 64 | int(lo)
        pts.update(x for x in (v - 1, v, v + 1) if 0 <= x < 1 << 128)
    q = S.from_ints(sorted(pts))
    from oracle.trie import Trie
    want = Trie(p, L, nh).lookup(q)
    reps = -(-(1 << 20) // q.shape[0])  # at least 2^20 lookups: the key-tops kernel runs
    q, want = np.tile(q, (reps, 1)), np.tile(want, reps)
    for kpl, R in ((fanout // 2, 2), (fanout // 4, 1)):
        try:
            P.planb_set_tuning(h, kpl, -1, R, 1024, 2)
        except P.PlanbError as e:
            assert e.code == P.PLANB_ERANGE
            continue
        say(f"wide tops fanout={fanout} kpl={kpl} R={R} n={q.shape[0]}")
        out = out_u16(q.shape[0])
        P.planb_lookup(h, to_dev(q), q.shape[0], out)
        assert np.array_equal(host_u16(out, q.shape[0]), want)
