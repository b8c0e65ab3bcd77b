// Host-side pre-computation of the PlanB lookup structure.
//
// Section 3 "From 2D Prefixes to 1D Intervals": every rule (P, L) becomes the
// address range [P, P + 2^(128-L) - 1]; the range boundaries split the address
// space into elementary intervals, each resolved once to its longest covering
// rule.  Section 3 "1D Search with Linearized B+-Tree" and Algorithm 2: the
// interval starts are the keys of a B+-tree stored level by level in one flat
// array.  Departures from the printed Algorithm 2 (each is a reading of a
// garbled or underspecified step, kept consistent with the paper's text):
//  * the end boundary is exclusive and computed on 129 bits (the algorithm
//    uses P + 2^(64-L) on 64 bits); an end of 2^128 produces no event;
//  * events are ordered by (address, END before START, START by ascending
//    length) so that the stack top after all events at one address is the
//    longest rule covering it;
//  * an interval at address 0 always exists (the default route, or NO_ROUTE);
//  * internal separators are the minimum key of each child's whole subtree
//    (the printed copy of "the child's first key" equals that only one level
//    above the leaves).
#include "builder.hpp"

#include <algorithm>

namespace planb {
namespace {

enum : uint8_t { kEnd = 0, kStart = 1 };

struct Event {
    U128 addr;
    uint8_t kind;
    uint8_t len;
    uint16_t nh;
};

// (hi, lo) with every bit below the top L bits cleared.
inline U128 mask_to(U128 p, int L)
{
    if (L == 0) return U128{0, 0};
    if (L <= 64) return U128{L == 64 ? p.hi : (p.hi & ~((~0ull) >> L)), 0};
    int h = 128 - L;  // host bits in lo, 0..63
    return U128{p.hi, h == 0 ? p.lo : (p.lo & ~((1ull << h) - 1))};
}

// start + 2^(128-L); returns false when the sum is 2^128 (no end boundary).
inline bool range_end(U128 start, int L, U128* end)
{
    if (L == 0) return false;
    int h = 128 - L;  // 0..127
    U128 r = start;
    if (h >= 64) {
        uint64_t add = 1ull << (h - 64);
        r.hi = start.hi + add;
        if (r.hi < start.hi) return false;
    } else {
        uint64_t add = 1ull << h;
        r.lo = start.lo + add;
        uint64_t carry = r.lo < start.lo ? 1 : 0;
        r.hi = start.hi + carry;
        if (carry && r.hi == 0) return false;
    }
    *end = r;
    return true;
}

}  // namespace

int make_intervals(const U128* prefixes, const uint8_t* lengths, const uint16_t* next_hops,
                   size_t n, bool merge_equal, Intervals* out, std::string* err)
{
    std::vector<Event> ev;
    ev.reserve(2 * n);
    for (size_t i = 0; i < n; ++i) {
        int L = lengths[i];
        if (L > 128) {
            *err = "prefix length " + std::to_string(L) + " > 128 at rule " + std::to_string(i);
            return -1;
        }
        if (next_hops[i] == kNoRoute) {
            *err = "next hop 0xFFFF (reserved for NO_ROUTE) at rule " + std::to_string(i);
            return -1;
        }
        U128 s = mask_to(prefixes[i], L);
        ev.push_back(Event{s, kStart, (uint8_t)L, next_hops[i]});
        U128 e;
        if (range_end(s, L, &e)) ev.push_back(Event{e, kEnd, (uint8_t)L, 0});
    }
    std::sort(ev.begin(), ev.end(), [](const Event& a, const Event& b) {
        if (a.addr != b.addr) return a.addr < b.addr;
        if (a.kind != b.kind) return a.kind < b.kind;  // END first
        return a.len < b.len;                          // shorter (outer) START first
    });
    for (size_t i = 1; i < ev.size(); ++i) {
        if (ev[i].kind == kStart && ev[i - 1].kind == kStart && ev[i].addr == ev[i - 1].addr &&
            ev[i].len == ev[i - 1].len) {
            *err = "duplicate rule after masking host bits";
            return -2;
        }
    }
    out->starts.clear();
    out->nh.clear();
    out->starts.reserve(ev.size() + 1);
    out->nh.reserve(ev.size() + 1);
    if (ev.empty() || ev[0].addr != U128{0, 0}) {
        out->starts.push_back(U128{0, 0});
        out->nh.push_back(kNoRoute);
    }
    std::vector<uint16_t> stack;
    stack.reserve(130);
    size_t i = 0;
    while (i < ev.size()) {
        U128 a = ev[i].addr;
        for (; i < ev.size() && ev[i].addr == a; ++i) {
            if (ev[i].kind == kStart) {
                stack.push_back(ev[i].nh);
            } else {
                if (stack.empty()) {
                    *err = "internal error: unbalanced interval sweep";
                    return -4;
                }
                stack.pop_back();
            }
        }
        uint16_t nh = stack.empty() ? kNoRoute : stack.back();
        if (merge_equal && !out->nh.empty() && out->nh.back() == nh) continue;
        out->starts.push_back(a);
        out->nh.push_back(nh);
    }
    return 0;
}

int plan_layout(uint64_t m, uint32_t b, uint32_t slots, uint32_t leaf_cap, uint32_t leaf_slots, bool trimmed,
                Layout* lay, std::string* err)
{
    if (b < 2 || slots < b - 1 || m == 0 || leaf_cap == 0 || leaf_slots < leaf_cap) {
        *err = "layout needs m >= 1, fanout >= 2, slots >= fanout - 1 and leaf slots >= leaf keys >= 1";
        return -1;
    }
    Layout L;
    L.b = b;
    L.slots = slots;
    L.leaf_cap = leaf_cap;
    L.leaf_slots = leaf_slots;
    L.m = m;
    L.leaves = (m + leaf_cap - 1) / leaf_cap;
    // smallest D with leaf_cap * b^(D-1) >= m
    uint32_t D = 1;
    uint64_t cap = leaf_cap;
    while (cap < m) {
        if (D >= (uint32_t)kMaxLevels) {
            *err = "tree deeper than the supported maximum";
            return -5;
        }
        cap *= b;
        ++D;
    }
    L.depth = D;
    L.nodes[D - 1] = L.leaves;
    uint64_t span = 1;  // leaves under one node of the level being sized
    for (int l = (int)D - 2; l >= 0; --l) {
        span *= b;
        if (trimmed) {
            L.nodes[l] = (L.leaves + span - 1) / span;
        } else {  // complete level: b^l nodes
            uint64_t full = 1;
            for (int t = 0; t < l; ++t) full *= b;
            L.nodes[l] = full;
        }
    }
    L.offset[0] = 0;
    for (uint32_t l = 0; l < D; ++l) L.offset[l + 1] = L.offset[l] + L.nodes[l];
    *lay = L;
    return 0;
}

void fill_keys(const Intervals& iv, const Layout& lay, int key_bytes, std::vector<U128>* keys)
{
    const uint64_t b = lay.b, S = lay.slots, k = b - 1, D = lay.depth, m = iv.starts.size();
    const uint64_t LC = lay.leaf_cap, LS = lay.leaf_slots;
    keys->assign(lay.total_slots(), kSentinel);
    U128* K = keys->data();
    const uint64_t leaf0 = lay.leaf_base();
    for (uint64_t i = 0; i < m; ++i) K[leaf0 + (i / LC) * LS + leaf_key_slot((uint32_t)(i % LC), key_bytes)] = iv.starts[i];
    // internal levels: separator j-1 of node q = first key of the leftmost
    // leaf under child q*b + j
    uint64_t span = 1;  // leaves under one node of level l + 1
    for (int l = (int)D - 2; l >= 0; --l) {
        for (uint64_t q = 0; q < lay.nodes[l]; ++q) {
            for (uint64_t j = 1; j <= k; ++j) {
                uint64_t leaf = (q * b + j) * span;
                if (leaf < lay.leaves) K[(lay.offset[l] + q) * S + (j - 1)] = iv.starts[leaf * LC];
            }
        }
        span *= b;
    }
}

}  // namespace planb
