// Host-side pre-computation: range conversion, elementary intervals and the
// linearized B+-tree key array (Section 3 of the PlanB paper, Algorithm 2).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "leaf_format.hpp"

namespace planb {

struct U128 {
    uint64_t hi, lo;
};

inline bool operator<(U128 a, U128 b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }
inline bool operator==(U128 a, U128 b) { return a.hi == b.hi && a.lo == b.lo; }
inline bool operator!=(U128 a, U128 b) { return !(a == b); }
inline bool operator<=(U128 a, U128 b) { return !(b < a); }

constexpr U128 kSentinel{~0ull, ~0ull};  // padding key, 2^128 - 1
constexpr uint16_t kNoRoute = 0xFFFFu;
constexpr int kMaxLevels = 16;

// Elementary intervals: starts strictly increasing, starts[0] == 0; the
// interval i covers [starts[i], starts[i+1]) (the last one runs to 2^128 - 1).
struct Intervals {
    std::vector<U128> starts;
    std::vector<uint16_t> nh;
};

// Status codes mirror planb_status_t.
int make_intervals(const U128* prefixes, const uint8_t* lengths, const uint16_t* next_hops,
                   size_t n, bool merge_equal, Intervals* out, std::string* err);

// Shape of a tree over m keys: internal nodes of fanout b with `slots` key
// slots each; leaves of `leaf_slots` slots holding `leaf_cap` keys each.
struct Layout {
    uint32_t b = 0, slots = 0, depth = 0;
    uint32_t leaf_cap = 0, leaf_slots = 0;
    uint64_t m = 0, leaves = 0;
    uint64_t nodes[kMaxLevels] = {};       // nodes per level, the leaf level last
    uint64_t offset[kMaxLevels + 1] = {};  // first node of each level (internal levels, then leaves)
    uint64_t internal_nodes() const { return offset[depth - 1]; }
    // slot of leaf 0's first key: the internal slots rounded up to a whole leaf,
    // so that leaves of 128 bytes never straddle a cache line
    uint64_t leaf_base() const { return (internal_nodes() * slots + leaf_slots - 1) / leaf_slots * leaf_slots; }
    uint64_t total_slots() const { return leaf_base() + leaves * leaf_slots; }
    // slots occupied by the top `levels` levels (the whole array when levels = depth)
    uint64_t prefix_slots(uint32_t levels) const { return levels >= depth ? total_slots() : offset[levels] * slots; }
};

// trimmed: drop trailing internal nodes holding only sentinels.
int plan_layout(uint64_t m, uint32_t b, uint32_t slots, uint32_t leaf_cap, uint32_t leaf_slots, bool trimmed,
                Layout* lay, std::string* err);

// Fills the slot array (every unused slot is the sentinel 2^128 - 1).  Leaf q
// holds the interval starts q*leaf_cap ..; its key s sits in slot s, or, with
// key_bytes = 8, where the blocked 64-bit leaf format puts it.  Separator j-1
// of an internal node is the smallest key under its child j.
void fill_keys(const Intervals& iv, const Layout& lay, int key_bytes, std::vector<U128>* keys);

}  // namespace planb
