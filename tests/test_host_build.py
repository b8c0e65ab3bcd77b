"""Host-side steps of the build, checked on the CPU (no GPU needed).

* elementary intervals (range conversion + sweep) against the brute-force
  oracle's LPM at every interval's first and last address;
* interval invariants (partition of the address space, m <= 2n + 1, every rule
  boundary present);
* the paper's worked range-conversion example;
* build errors (length > 128, reserved next hop, duplicates after masking);
* layout arithmetic against the paper's capacity numbers and closed forms;
* the key array: sentinel slots, leaves in order, separators = subtree minima,
  and a host re-run of the count-based descent == textbook predecessor search.
"""
import bisect
import ipaddress
import os

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

import planb_synth as S
from oracle.brute import NO_ROUTE, lpm_bruteforce, lpm_one, rules_of
from paper_2604_14650_amd import planb as P
from test_oracle_pins import fibs, fib_arrays, GOLDEN

M128 = (1 << 128) - 1


def ints(a):
    return [S.to_int(r) for r in a]


def check_intervals(rules, merge=False):
    p, L, nh = fib_arrays(rules)
    starts, inh = P.planb_build_intervals(p, L, nh, flags=P.PLANB_FLAG_MERGE_EQUAL_NH if merge else 0)
    s = ints(starts)
    m = len(s)
    assert s[0] == 0
    assert all(s[i] < s[i + 1] for i in range(m - 1))
    assert m <= 2 * len(rules) + 1
    if not merge:
        bounds = set()
        for Pv, Lv, _ in rules:
            bounds.add(Pv)
            e = Pv + (1 << (128 - Lv))
            if e <= M128:
                bounds.add(e)
        assert bounds <= set(s)
    else:
        assert all(inh[i] != inh[i + 1] for i in range(m - 1))
    for i in range(m):
        last = (s[i + 1] - 1) if i + 1 < m else M128
        assert lpm_one(s[i], rules) == inh[i]
        assert lpm_one(last, rules) == inh[i]
    return s, inh


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(fibs(max_rules=14), st.booleans())
def test_intervals_match_oracle(rules, merge):
    check_intervals(rules, merge)


def test_intervals_on_tiny_workload():
    fib = S.make_fib(S.TINY, 11)
    rules = rules_of(fib.prefixes, fib.lengths, fib.next_hops)
    s, inh = check_intervals(rules)
    # every rule boundary splits the space once: nothing merged away
    assert len(s) <= 2 * len(rules) + 1
    # random addresses: predecessor interval's next hop == LPM
    a = S.tiny_traffic(fib, 2000, seed=5)
    want = lpm_bruteforce(fib.prefixes, fib.lengths, fib.next_hops, a)
    got = [inh[bisect.bisect_right(s, x) - 1] for x in ints(a)]
    assert list(want) == got


def test_worked_example_boundaries():
    with open(os.path.join(GOLDEN, "range_conversion.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            net, first, last = line.split()
            net = ipaddress.IPv6Network(net)
            first = int(ipaddress.IPv6Address(first))
            last = int(ipaddress.IPv6Address(last))
            p, L, nh = fib_arrays([(int(net.network_address), net.prefixlen, 3)])
            starts, inh = P.planb_build_intervals(p, L, nh)
            assert ints(starts) == [0, first, last + 1]
            assert list(inh) == [NO_ROUTE, 3, NO_ROUTE]


def test_top_of_space_has_no_end_boundary():
    rules = [(0, 0, 1), (0xFFFF << 112, 16, 2), (M128, 128, 3)]
    s, inh = check_intervals(rules)
    assert s == [0, 0xFFFF << 112, M128]
    assert list(inh) == [1, 2, 3]


def test_host_bits_are_masked():
    p = S.from_ints([(0x20010DB8 << 96) | 0xABCDEF])
    starts, _ = P.planb_build_intervals(p, np.array([32], np.uint8), np.array([5], np.uint16))
    assert ints(starts) == [0, 0x20010DB8 << 96, 0x20010DB9 << 96]


def test_empty_fib_is_one_no_route_interval():
    starts, inh = P.planb_build_intervals(np.zeros((0, 2), np.uint64), np.zeros(0, np.uint8),
                                          np.zeros(0, np.uint16))
    assert ints(starts) == [0] and list(inh) == [NO_ROUTE]


@pytest.mark.parametrize("lengths,nhs,code", [
    ([129], [1], P.PLANB_EINVAL),
    ([32], [0xFFFF], P.PLANB_EINVAL),
])
def test_build_rejects_bad_rules(lengths, nhs, code):
    p = S.from_ints([0x2001 << 112] * len(lengths))
    with pytest.raises(P.PlanbError) as e:
        P.planb_build_intervals(p, np.array(lengths, np.uint8), np.array(nhs, np.uint16))
    assert e.value.code == code


def test_build_rejects_duplicates_after_masking():
    p = S.from_ints([0x2001 << 112, (0x2001 << 112) | 77])
    with pytest.raises(P.PlanbError) as e:
        P.planb_build_intervals(p, np.array([16, 16], np.uint8), np.array([1, 2], np.uint16))
    assert e.value.code == P.PLANB_EDUP


# ---------------------------------------------------------------- layout pins
def _golden_layout():
    d = {}
    with open(os.path.join(GOLDEN, "layout_capacity.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                k, v = line.split("=")
                d[k] = float(v) if "." in v else int(v)
    return d


def test_layout_matches_paper_capacity_numbers():
    g = _golden_layout()
    b, k, kb = g["fanout"], g["keys_per_node"], g["key_bytes"]
    MiB = 1 << 20
    lay = P.planb_layout(g["keys_a"], b, k, trimmed=False)
    assert lay["depth"] == g["internal_levels_a"] + 1
    assert lay["level_nodes"][-1] == g["leaves_a"]
    assert lay["level_offset"][-2] == g["internal_nodes_a"]
    assert g["leaves_a"] * k == g["keys_a"]
    leaf_bytes = g["leaves_a"] * k * kb
    internal_bytes = lay["level_offset"][-2] * k * kb
    assert round(leaf_bytes / MiB, 1) == g["leaf_mib_a"]
    assert round(internal_bytes / MiB, 2) == g["internal_mib_a"]
    # two intervals per prefix -> bytes per prefix
    assert round((leaf_bytes + internal_bytes) / (g["keys_a"] / 2)) == g["bytes_per_prefix_a"]
    # one more key no longer fits five internal levels
    assert P.planb_layout(g["keys_a"] + 1, b, k, trimmed=False)["depth"] == g["internal_levels_a"] + 2
    lay_b = P.planb_layout(g["keys_b"], b, k, trimmed=False)
    assert lay_b["depth"] == g["internal_levels_b"] + 1 == g["accesses_b"]
    assert round(lay_b["level_nodes"][-1] * k * kb / MiB) == g["leaf_mib_b"]
    assert round(lay_b["level_offset"][-2] * k * kb / MiB) == g["internal_mib_b"]
    # root keys at 0..7, the children's first key at index 8
    assert lay["level_offset"][0] * k == g["root_first_key"]
    assert lay["level_offset"][1] * k - 1 == g["root_last_key"]
    assert lay["level_offset"][1] * k == g["children_first_key"]


@pytest.mark.parametrize("b", [3, 9, 16, 17])
def test_level_start_and_child_start_closed_forms(b):
    """level_start(d) = k (b^d - 1)/(b - 1) and child_start(d, j, c) =
    level_start(d+1) + (j b + c) k; Listing 1's recurrence i' = (k+1) i + (c+1) k
    reaches the same index from node start i = level_start(d) + j k."""
    k = b - 1
    lay = P.planb_layout(k * b ** 5, b, k, trimmed=False)
    for d in range(lay["depth"]):
        assert lay["level_offset"][d] * k == k * (b ** d - 1) // (b - 1)
    for d in range(4):
        ls1 = lay["level_offset"][d + 1] * k
        for j in (0, 1, b ** d - 1):
            i = lay["level_offset"][d] * k + j * k
            for c in range(b):
                assert (k + 1) * i + (c + 1) * k == ls1 + (j * b + c) * k


@pytest.mark.parametrize("m,b", [(1, 16), (15, 16), (16, 16), (1000, 8), (4096, 16), (70000, 32)])
def test_trimmed_layout_depth(m, b):
    lay = P.planb_layout(m, b, b, trimmed=True)
    k = b - 1
    D = lay["depth"]
    assert k * b ** (D - 1) >= m and (D == 1 or k * b ** (D - 2) < m)
    leaves = -(-m // k)
    assert lay["level_nodes"][-1] == leaves
    for l in range(D - 1):
        assert lay["level_nodes"][l] == -(-leaves // b ** (D - 1 - l))


# ------------------------------------------------------------- key array
# Leaves of a FIB with 128-bit keys: max(b slots, 128 bytes) long, holding as
# many 16-byte keys plus 2-byte next hops as fit (written out per fanout).
LEAF_SHAPE_128 = {8: (7, 8), 16: (14, 16), 32: (28, 32)}  # b -> (keys, slots)


def _descend(keys, info, x):
    """Count-based descent over the host key array (the semantics the kernel
    implements): c = #{keys <= x}, child q*b + c clamped to the level's last
    node; at leaf q with L keys the interval is q*L + c - 1 (clamped to m-1)."""
    b, D = info["fanout"], info["depth"]
    off, nodes = info["level_offset"], info["level_nodes"]
    L, LS, base = info["leaf_keys"], info["leaf_slots"], info["leaf_base"]
    q = 0
    for l in range(D - 1):
        node = (off[l] + q) * b
        c = sum(1 for s in range(b) if keys[node + s] <= x)
        q = min(q * b + c, nodes[l + 1] - 1)
    leaf = base + q * LS
    c = sum(1 for s in range(L) if keys[leaf + s] <= x)
    return min(q * L + c - 1, info["intervals"] - 1)


@pytest.mark.parametrize("b", [8, 16, 32])
@pytest.mark.parametrize("m", [1, 2, 7, 15, 16, 17, 300, 4000])
def test_key_array_structure_and_descent(b, m):
    rng = np.random.default_rng(m * 100 + b)
    vals = sorted(set(int(v) for v in rng.integers(1, 2**62, size=m - 1)) | {0})
    vals = sorted(set(vals) | {0})
    while len(vals) < m:
        vals.append(vals[-1] + 1)
    vals = [v << 64 | (v * 7 & 0xFFFF) for v in vals[:m]]
    vals[0] = 0
    starts = S.from_ints(vals)
    keys_arr, info = P.planb_build_keys(starts, b)
    keys = ints(keys_arr)
    D, off, nodes = info["depth"], info["level_offset"], info["level_nodes"]
    L, LS, base = info["leaf_keys"], info["leaf_slots"], info["leaf_base"]
    assert (L, LS) == LEAF_SHAPE_128[b]
    leaves = -(-m // L)
    assert nodes[D - 1] == leaves
    # leaves start at the first whole leaf after the internal nodes
    assert base % LS == 0 and off[D - 1] * b <= base < off[D - 1] * b + LS
    assert len(keys) == base + leaves * LS
    k = b - 1
    for q in range(off[D - 1]):
        assert keys[q * b + k] == M128  # sentinel slot of every internal node
    assert all(keys[s] == M128 for s in range(off[D - 1] * b, base))  # alignment gap
    leaf_keys = [keys[base + (i // L) * LS + i % L] for i in range(m)]
    assert leaf_keys == vals
    for q in range(leaves):  # unused key slots and the next-hop area hold sentinels here
        used = min(L, m - q * L)
        assert all(keys[base + q * LS + s] == M128 for s in range(used, LS))

    def subtree_min(l, q):
        while l < D - 1:
            l, q = l + 1, q * b
        return keys[base + q * LS] if q < leaves else M128

    for l in range(D - 1):
        for q in range(nodes[l]):
            for j in range(1, b):
                child = q * b + j
                want = subtree_min(l + 1, child) if child < nodes[l + 1] else M128
                assert keys[(off[l] + q) * b + j - 1] == want
    probes = [0, 1, M128, M128 - 1] + vals + [v - 1 for v in vals[1:]] + [v + 1 for v in vals]
    probes += [int(x) << 64 for x in rng.integers(0, 2**62, size=200)]
    for x in probes:
        assert _descend(keys, info, x) == bisect.bisect_right(vals, x) - 1


def test_descent_with_top_key_equal_to_sentinel():
    vals = [0, 5, M128]
    keys_arr, info = P.planb_build_keys(S.from_ints(vals), 8)
    keys = ints(keys_arr)
    for x, want in [(0, 0), (4, 0), (5, 1), (M128 - 1, 1), (M128, 2)]:
        assert _descend(keys, info, x) == want


# ------------------------------------------------------------- device image
# (keys, slots) per leaf of a FIB's device image, written out per key width and
# fanout: 64-bit slots: 32-byte blocks of 3 keys + their 3 next hops; 128-bit
# slots: the keys, then their next hops.
LEAF_SHAPE = {(32, 8): (20, 32), (32, 16): (20, 32), (32, 32): (20, 32),
              (64, 8): (12, 16), (64, 16): (12, 16), (64, 32): (24, 32),
              (128, 8): (7, 8), (128, 16): (14, 16), (128, 32): (28, 32)}


def _leaf_key_off(s, kbits, L):
    if kbits == 32:  # 32-byte blocks of five keys, then their five hops
        return (s // 5) * 32 + (s % 5) * 4
    return (s // 3) * 32 + (s % 3) * 8 if kbits == 64 else 16 * s


def _leaf_hop_off(s, kbits, L):
    if kbits == 32:
        return (s // 5) * 32 + 20 + (s % 5) * 2
    return (s // 3) * 32 + 24 + (s % 3) * 2 if kbits == 64 else 16 * L + 2 * s


def _slot_key(img, slot, kbits):
    """Key in a slot of the image as a 128-bit integer (narrow slots hold the top bits)."""
    if kbits == 32:
        return int.from_bytes(img[4 * slot:4 * slot + 4].tobytes(), "little") << 96
    if kbits == 64:
        return int.from_bytes(img[8 * slot:8 * slot + 8].tobytes(), "little") << 64
    hi = int.from_bytes(img[16 * slot:16 * slot + 8].tobytes(), "little")
    lo = int.from_bytes(img[16 * slot + 8:16 * slot + 16].tobytes(), "little")
    return hi << 64 | lo


def _image_lookup(img, info, x):
    """Descent over the byte image, as the kernel does it: (interval index, next hop)."""
    b, D, kbits = info["fanout"], info["depth"], info["key_bits"]
    off, nodes = info["level_offset"], info["level_nodes"]
    L, LS, base = info["leaf_keys"], info["leaf_slots"], info["leaf_base"]
    kb = kbits // 8
    xk = x if kbits == 128 else (x >> (128 - kbits)) << (128 - kbits)  # narrow keys compare the top bits
    q = 0
    for l in range(D - 1):
        c = sum(1 for s in range(b) if _slot_key(img, (off[l] + q) * b + s, kbits) <= xk)
        q = min(q * b + c, nodes[l + 1] - 1)
    leaf = (base + q * LS) * kb
    keys = [_key_at(img, leaf + _leaf_key_off(s, kbits, L), kbits) for s in range(L)]
    c = sum(1 for k in keys if k <= xk)
    idx = min(q * L + c - 1, info["intervals"] - 1)
    pos = idx - q * L
    hop = int.from_bytes(img[leaf + _leaf_hop_off(pos, kbits, L):][:2].tobytes(), "little")
    return idx, hop


def _key_at(img, byte, kbits):
    if kbits == 32:
        return int.from_bytes(img[byte:byte + 4].tobytes(), "little") << 96
    if kbits == 64:
        return int.from_bytes(img[byte:byte + 8].tobytes(), "little") << 64
    return (int.from_bytes(img[byte:byte + 8].tobytes(), "little") << 64 |
            int.from_bytes(img[byte + 8:byte + 16].tobytes(), "little"))


@pytest.mark.parametrize("b", [8, 16, 32])
@pytest.mark.parametrize("kbits", [32, 64, 128])
@pytest.mark.parametrize("m", [1, 2, 11, 12, 13, 19, 20, 21, 25, 700, 5000])
def test_device_image_structure_and_descent(b, kbits, m):
    rng = np.random.default_rng(7 * m + b + kbits)
    top = 31 if kbits == 32 else 63
    his = sorted(set(int(v) for v in rng.integers(1, 2**top, size=m - 1)) | {0})
    while len(his) < m:
        his.append(his[-1] + 1)
    his = his[:m]
    if kbits == 32:
        vals = [h << 96 for h in his]
    else:
        lo_mask = 0 if kbits == 64 else 0xFFFF
        vals = [h << 64 | (h * 13 & lo_mask) for h in his]
    vals[0] = 0
    nh = rng.integers(0, 0xFFFF, size=m).astype(np.uint16)
    img, info = P.planb_build_image(S.from_ints(vals), nh, b, kbits)
    assert info["key_bits"] == kbits and info["intervals"] == m
    L, LS, base = info["leaf_keys"], info["leaf_slots"], info["leaf_base"]
    assert (L, LS) == LEAF_SHAPE[(kbits, b)]
    kb = kbits // 8
    leaves = -(-m // L)
    assert info["level_nodes"][-1] == leaves
    assert LS * kb >= 128 and base % LS == 0 and len(img) == (base + leaves * LS) * kb == info["key_bytes"]
    for q in range(leaves):
        leaf = (base + q * LS) * kb
        for s in range(L):
            i = q * L + s
            key = _key_at(img, leaf + _leaf_key_off(s, kbits, L), kbits)
            hop = int.from_bytes(img[leaf + _leaf_hop_off(s, kbits, L):][:2].tobytes(), "little")
            if i < m:
                assert key == vals[i] and hop == nh[i], (q, s)
            else:
                assert key == M128 >> (128 - kbits) << (128 - kbits) and hop == 0xFFFF
    probes = [0, 1, M128, M128 - 1] + vals + [v - 1 for v in vals[1:]] + [v + 1 for v in vals]
    probes += [int(x) << 64 | int(y) for x, y in zip(rng.integers(0, 2**63, size=100), rng.integers(0, 2**63, size=100))]
    for x in probes[:1500]:
        want = bisect.bisect_right(vals, x) - 1
        assert _image_lookup(img, info, x) == (want, int(nh[want])), hex(x)


def test_device_image_key_width_choice():
    vals = [0, 5 << 64, 9 << 64 | 1]
    nh = np.array([1, 2, 3], np.uint16)
    _, info = P.planb_build_image(S.from_ints(vals), nh, 8, 0)
    assert info["key_bits"] == 128  # a start with a nonzero low word
    _, info = P.planb_build_image(S.from_ints(vals[:2]), nh[:2], 8, 0)
    assert info["key_bits"] == 64  # nonzero bits below the top 32
    _, info = P.planb_build_image(S.from_ints([0, 5 << 96]), nh[:2], 8, 0)
    assert info["key_bits"] == 32  # only the top 32 bits are ever nonzero
    for kb in (64, 128):
        _, info = P.planb_build_image(S.from_ints([0, 5 << 96]), nh[:2], 8, kb)
        assert info["key_bits"] == kb
    with pytest.raises(P.PlanbError):
        P.planb_build_image(S.from_ints(vals), nh, 8, 64)
    with pytest.raises(P.PlanbError):
        P.planb_build_image(S.from_ints(vals[:2]), nh[:2], 8, 32)
    with pytest.raises(P.PlanbError):
        P.planb_build_image(S.from_ints([1, 2]), nh[:2], 8, 0)  # starts[0] must be 0


# ------------------------------------------------------------- CPU baseline
@pytest.mark.parametrize("b", [8, 16, 32])
@pytest.mark.parametrize("key_bits", [0, 128])
def test_cpu_btree_baseline_ipv4(b, key_bits):
    """The CPU baseline on an IPv4 FIB (32-bit key slots when automatic)."""
    from oracle.trie import Trie
    fib = S.make_fib(S.IPV4_TINY, 40 + b)
    a4 = S.ipv4_traffic(fib, 20000, 0.7, 3 + b)
    addrs = np.concatenate([S.v4_as_128(a4), S.from_ints([0, (1 << 128) - 1, 0xFFFFFFFF << 96])])
    tree = P.CpuTree(fib.prefixes, fib.lengths, fib.next_hops, fanout=b, key_bits=key_bits)
    assert tree.shape["key_bits"] == (key_bits or 32)
    want = Trie(fib.prefixes, fib.lengths, fib.next_hops).lookup(addrs)
    assert np.array_equal(tree.lookup(addrs, 2), want)


@pytest.mark.parametrize("b", [8, 16, 32])
@pytest.mark.parametrize("key_bits", [0, 128])
def test_cpu_btree_baseline_matches_oracle(b, key_bits):
    """The host-core linearized B+-tree (planb_cpu_lookup over the device image)
    returns the oracle's next hops."""
    from oracle.trie import Trie
    fib = S.make_fib(S.vrf_spec(3000), 31 + b)
    addrs = S.mixed_traffic(fib, 20000, 0.5, 7 + b)
    addrs = np.concatenate([addrs, S.from_ints([0, 1, (1 << 128) - 1, (1 << 128) - 2])])
    tree = P.CpuTree(fib.prefixes, fib.lengths, fib.next_hops, fanout=b, key_bits=key_bits)
    assert tree.shape["key_bits"] == (key_bits or 64)
    want = Trie(fib.prefixes, fib.lengths, fib.next_hops).lookup(addrs)
    for threads in (1, 3):
        assert np.array_equal(tree.lookup(addrs, threads), want)


@pytest.mark.parametrize("kind", ["vrf", "large_slice", "tiny"])
@pytest.mark.parametrize("key_bits", [64, 128])
def test_paper_cpu_tree_matches_oracle(kind, key_bits):
    """The paper-design CPU baseline (fanout 9, 8 keys per node, vector
    compare + popcount) returns the oracle's next hops, with 64-bit keys where
    every start's low word is zero and with 128-bit keys; /128 host routes
    need (and get) 128-bit keys."""
    from oracle.trie import Trie
    if kind == "vrf":
        fib = S.make_fib(S.vrf_spec(5000), 71)
    elif kind == "tiny":
        fib = S.make_fib(S.TINY, 11)
    else:  # a slice of the 1M-prefix recipe: /128 host routes included
        big = S.make_fib(S.LARGE, 33)
        keep = np.arange(0, len(big), 97)
        fib = S.Fib(big.prefixes[keep], big.lengths[keep], big.next_hops[keep])
    rng = np.random.default_rng(5)
    addrs = S.mixed_traffic(fib, 30000, 0.6, 9)
    starts, _ = P.planb_build_intervals(fib.prefixes, fib.lengths, fib.next_hops)
    around = starts[rng.integers(0, len(starts), 2000)]
    below = around.copy()  # each start - 1 (128-bit)
    borrow = below[:, 1] == 0
    below[:, 1] -= np.uint64(1)
    below[:, 0] -= borrow.astype(np.uint64)
    addrs = np.concatenate([addrs, around, below, S.from_ints([0, 1, (1 << 128) - 1, (1 << 128) - 2])])
    want = Trie(fib.prefixes, fib.lengths, fib.next_hops).lookup(addrs)
    lo_zero = bool(np.all(starts[:, 1] == 0))
    if key_bits == 64 and not lo_zero:
        with pytest.raises(P.PlanbError):
            P.PaperCpuTree(fib.prefixes, fib.lengths, fib.next_hops, key_bits=64)
        return
    tree = P.PaperCpuTree(fib.prefixes, fib.lengths, fib.next_hops, key_bits=key_bits)
    assert tree.isa in ("avx512", "avx2")
    assert 8 * 9 ** (tree.depth - 1) >= len(starts) and (tree.depth == 1 or 8 * 9 ** (tree.depth - 2) < len(starts))
    for threads in (1, 3):
        assert np.array_equal(tree.lookup(addrs, threads), want)
