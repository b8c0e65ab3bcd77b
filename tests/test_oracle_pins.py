"""Pins for the CPU oracle, against things other than the oracle itself.

* Python's ``ipaddress`` library (an independent implementation of "address x
  lies in network P/L") decides every match on small random FIBs.
* The paper's worked range-conversion example fixes where a /32 begins and ends.
* Closed-form special cases: an empty FIB, ::/0 alone, a /128 at the very top
  of the address space, ffff::/16 (whose range ends at 2^128 - 1).
* The trie and the brute force are two unrelated programs; they must agree.
* Planted mistakes in a copy of the brute force must be caught by these pins.
"""
import ipaddress
import os

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

import planb_synth as S
from oracle.brute import NO_ROUTE, lpm_bruteforce, lpm_bruteforce_np, lpm_one
from oracle.trie import Trie, lpm_trie

M128 = (1 << 128) - 1
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def mask(v, L):
    return v & ((M128 << (128 - L)) & M128)


def arr(vals):
    return S.from_ints(vals)


def fib_arrays(rules):
    """rules: list of (prefix_int, len, nh) -> (prefixes, lengths, next_hops)."""
    p = arr([r[0] for r in rules]) if rules else np.zeros((0, 2), dtype=np.uint64)
    L = np.array([r[1] for r in rules], dtype=np.uint8)
    nh = np.array([r[2] for r in rules], dtype=np.uint16)
    return p, L, nh


def ipaddress_lpm(rules, x):
    """Longest match decided by ipaddress membership tests only."""
    a = ipaddress.IPv6Address(x)
    best_len, best = -1, NO_ROUTE
    for P, L, nh in rules:
        if a in ipaddress.IPv6Network((P, L)) and L > best_len:
            best_len, best = L, nh
    return best


INTERESTING = [0, M128, 0x20010DB8 << 96, (0x20010DB8 << 96) | (1 << 80), 1 << 127,
               (1 << 127) - 1, 0xFFFF << 112, 0x2000 << 112, 0x3FFF << 112]


@st.composite
def fibs(draw, max_rules=10):
    """Small FIBs with nesting chains, adjacent siblings, shared starts and the
    special prefixes ::/0, /128 and ffff::/16."""
    rules = {}
    n = draw(st.integers(0, max_rules))
    for _ in range(n):
        kind = draw(st.sampled_from(["rand", "nest", "sibling", "same", "special"]))
        if kind == "special":
            P, L = draw(st.sampled_from([(0, 0), (M128, 128), (0xFFFF << 112, 16), (0, 128), (0, 1)]))
        elif kind in ("nest", "sibling", "same") and rules:
            Pp, Lp = draw(st.sampled_from(sorted(rules)))
            if kind == "nest":
                L = draw(st.integers(Lp, 128))
                P = mask(Pp | (draw(st.integers(0, M128)) & (M128 >> Lp if Lp else M128)), L)
            elif kind == "same":
                L = draw(st.integers(0, 128))
                P = mask(Pp, L)
            else:  # the adjacent range of the same length
                P = mask((Pp + (1 << (128 - Lp))) & M128, Lp) if Lp else 0
                L = Lp
        else:
            L = draw(st.sampled_from([1, 3, 16, 29, 32, 48, 63, 64, 65, 96, 127, 128]) | st.integers(0, 128))
            P = mask(draw(st.sampled_from(INTERESTING) | st.integers(0, M128)), L)
        rules.setdefault((P, L), draw(st.integers(0, 65534)))
    return [(P, L, nh) for (P, L), nh in rules.items()]


def queries_for(rules, extra=()):
    q = {0, M128, *extra}
    for P, L, _ in rules:
        end = P + (1 << (128 - L)) - 1
        for v in (P - 1, P, P + 1, end - 1, end, end + 1):
            if 0 <= v <= M128:
                q.add(v)
    return sorted(q)


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(fibs(), st.lists(st.integers(0, M128), max_size=5))
def test_bruteforce_matches_ipaddress_membership(rules, extra):
    for x in queries_for(rules, extra):
        assert lpm_one(x, rules) == ipaddress_lpm(rules, x), hex(x)


@settings(max_examples=300, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(fibs(max_rules=14), st.lists(st.integers(0, M128), max_size=5))
def test_trie_matches_bruteforce(rules, extra):
    p, L, nh = fib_arrays(rules)
    qs = arr(queries_for(rules, extra))
    want = lpm_bruteforce(p, L, nh, qs)
    assert np.array_equal(lpm_trie(p, L, nh, qs, nthreads=2), want)
    assert np.array_equal(lpm_bruteforce_np(p, L, nh, qs), want)


def _parse_golden_range():
    rows = []
    with open(os.path.join(GOLDEN, "range_conversion.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            net, first, last = line.split()
            rows.append((ipaddress.IPv6Network(net), int(ipaddress.IPv6Address(first)),
                         int(ipaddress.IPv6Address(last))))
    return rows


def test_worked_example_range_edges():
    """The paper's /32 example: every address of [start, end] matches the rule,
    the neighbours just outside it do not."""
    for net, first, last in _parse_golden_range():
        rules = [(int(net.network_address), net.prefixlen, 7)]
        p, L, nh = fib_arrays(rules)
        qs = arr([first - 1, first, first + 12345, last - 1, last, last + 1])
        want = [NO_ROUTE, 7, 7, 7, 7, NO_ROUTE]
        assert list(lpm_bruteforce(p, L, nh, qs)) == want
        assert list(lpm_trie(p, L, nh, qs)) == want


def test_closed_form_special_cases():
    qs = arr([0, 1, 1 << 64, (1 << 127), M128 - 1, M128])
    empty = fib_arrays([])
    assert list(lpm_trie(*empty, qs)) == [NO_ROUTE] * 6
    assert list(lpm_bruteforce(*empty, qs)) == [NO_ROUTE] * 6
    default = fib_arrays([(0, 0, 9)])
    assert list(lpm_trie(*default, qs)) == [9] * 6
    top = fib_arrays([(M128, 128, 4), (0xFFFF << 112, 16, 5), (0, 0, 1)])
    want = [1, 1, 1, 1, 5, 4]
    assert list(lpm_trie(*top, qs)) == want
    assert list(lpm_bruteforce(*top, qs)) == want


def test_nested_chain_and_shared_start():
    base = 0x20010DB8 << 96
    rules = [(base, 32, 1), (base, 48, 2), (base, 64, 3), (base | (5 << 60), 68, 4), (0, 0, 0)]
    p, L, nh = fib_arrays(rules)
    qs = arr([base, base | (1 << 70), base | (1 << 65), base | (5 << 60) | 9, base | (1 << 90),
              (base + (1 << 96)), base - 1])
    want = [3, 2, 2, 4, 1, 0, 0]
    assert list(lpm_bruteforce(p, L, nh, qs)) == want
    assert list(lpm_trie(p, L, nh, qs)) == want


def test_trie_equals_numpy_bruteforce_on_tiny_workload():
    fib = S.make_fib(S.TINY, 11)
    a = S.tiny_traffic(fib, 4000, seed=3)
    assert np.array_equal(lpm_trie(fib.prefixes, fib.lengths, fib.next_hops, a),
                          lpm_bruteforce_np(fib.prefixes, fib.lengths, fib.next_hops, a))


def test_trie_thread_count_does_not_change_results():
    fib = S.make_fib(S.TINY, 12)
    a = S.tiny_traffic(fib, 20000, seed=4)
    t = Trie(fib.prefixes, fib.lengths, fib.next_hops)
    r1 = t.lookup(a, 1)
    for k in (2, 3, 7, 16):
        assert np.array_equal(t.lookup(a, k), r1)
    assert t.lookup(a[:0]).shape == (0,)


def test_trie_rejects_bad_length():
    with pytest.raises(ValueError):
        Trie(arr([0]), np.array([129], dtype=np.uint8), np.array([1], dtype=np.uint16))


# --- planted mistakes: each mutant of the brute-force scan must fail a pin ---
def _mutant_shift_off_by_one(x, rules):
    best_len, best = -1, NO_ROUTE
    for P, L, nh in rules:
        s = max(0, 127 - L)
        if (x >> s) == (P >> s) and L > best_len:
            best_len, best = L, nh
    return best


def _mutant_shortest_wins(x, rules):
    best_len, best = 999, NO_ROUTE
    for P, L, nh in rules:
        if (x >> (128 - L)) == (P >> (128 - L)) and L < best_len:
            best_len, best = L, nh
    return best


def _mutant_default_never_matches(x, rules):
    best_len, best = -1, NO_ROUTE
    for P, L, nh in rules:
        if L > 0 and (x >> (128 - L)) == (P >> (128 - L)) and L > best_len:
            best_len, best = L, nh
    return best


def _mutant_low_half_ignored(x, rules):
    best_len, best = -1, NO_ROUTE
    for P, L, nh in rules:
        s = 128 - min(L, 64)
        if (x >> s) == (P >> s) and L > best_len:
            best_len, best = L, nh
    return best


@pytest.mark.parametrize("mutant", [_mutant_shift_off_by_one, _mutant_shortest_wins,
                                    _mutant_default_never_matches, _mutant_low_half_ignored])
def test_planted_mistakes_are_caught(mutant):
    base = 0x20010DB8 << 96
    rules = [(0, 0, 1), (base, 32, 2), (base, 48, 3), (base | (0xAB << 40), 120, 4),
             (M128, 128, 5), ((0x2001 << 112), 16, 6)]
    caught = False
    for x in queries_for(rules):
        if mutant(x, rules) != ipaddress_lpm(rules, x):
            caught = True
            break
    assert caught
