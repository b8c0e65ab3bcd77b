// Host-side pre-computation: range conversion, elementary intervals and the
// linearized B+-tree key array (Section 3 of the PlanB paper, Algorithm 2).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

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

// Shape of a tree over m keys: fanout b, `slots` key slots per node.
struct Layout {
    uint32_t b = 0, slots = 0, depth = 0;
    uint64_t m = 0, leaves = 0;
    uint64_t nodes[kMaxLevels] = {};
    uint64_t offset[kMaxLevels + 1] = {};
    uint64_t total_nodes() const { return offset[depth]; }
};

// trimmed: drop trailing internal nodes holding only sentinels.
int plan_layout(uint64_t m, uint32_t b, uint32_t slots, bool trimmed, Layout* lay, std::string* err);

// Fills the node-major key array (slots = b: k = b-1 keys + one sentinel slot
// per node).  Leaves hold the interval starts in order, k per node; separator
// j-1 of an internal node is the smallest key under its child j.
void fill_keys(const Intervals& iv, const Layout& lay, std::vector<U128>* keys);

}  // namespace planb
