// CPU linearized B+-tree in the paper's own layout and search, the host-core
// baseline that the GPU lookups are reported beside.
//
// Layout (Section 3 "1D Search with Linearized B+-Tree", "Parameter Tuning",
// "Separation of Keys and Values"): fanout b = 9, so a node holds k = 8 keys,
// one 64-byte cache line of 64-bit keys; levels are stored one after another,
// node-major, and a child is found arithmetically (child q*9 + c of node q),
// with no pointers.  Separators are the minima of the child subtrees.  Next
// hops live in a separate array indexed by the interval.  128-bit keys keep
// the same shape with the high and low words of a node in two lines (8 high
// words, then 8 low words).
//
// Search (Algorithm 1, Listing 1, "Vectorization and SIMD Acceleration",
// "Batching", "Branch-Free Traversal and Loop Unrolling"): at every node the
// keys <= x are counted with one vector compare and a popcount of its mask
// (AVX-512 when the host has it, else AVX2); the count is the child; the
// depth is a template parameter, so the level loop is fully unrolled; a batch
// of addresses descends level by level together, each next node prefetched as
// soon as its index is known, so that their cache misses overlap.  Threads
// split the address array.
//
// This runs on the host only (built with the host compiler; it uses no HIP).
// No GPU entry point calls it and it is no fallback for them.
#include <immintrin.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "../../include/planb.h"

namespace {

constexpr int kKeys = 8;     // keys per node (one 64-byte line of 64-bit keys)
constexpr int kFan = 9;      // children per internal node
constexpr int kBatch = 32;   // addresses descending together (measured best of 8..128)
constexpr int kMaxDepth = 12;

enum class Isa { avx512, avx2 };

struct Aligned {
    uint64_t* p = nullptr;
    ~Aligned() { std::free(p); }
    bool alloc(size_t words)
    {
        const size_t bytes = (words * 8 + 63) / 64 * 64;
        p = static_cast<uint64_t*>(std::aligned_alloc(64, bytes ? bytes : 64));
        return p != nullptr;
    }
};

}  // namespace

struct planb_cpu_tree {
    uint32_t key_bits = 64;  // 64: high words only; 128: high and low words
    uint32_t depth = 1;      // levels, the leaf level included
    uint64_t m = 0;
    uint64_t off[kMaxDepth] = {};   // first node of each level
    uint64_t last[kMaxDepth] = {};  // last node of each level (clamp)
    Aligned hi, lo;                 // hi[node * 8 + s]; lo likewise (128-bit keys)
    std::vector<uint16_t> nh;       // next hop of interval i
    Isa isa = Isa::avx2;
};

namespace {

using Tree = planb_cpu_tree;

// ---- keys <= x among a node's 8 keys
__attribute__((target("avx512f"))) inline uint32_t count512_64(const uint64_t* k, uint64_t x)
{
    const __m512i v = _mm512_load_si512(reinterpret_cast<const void*>(k));
    return (uint32_t)__builtin_popcount(_mm512_cmple_epu64_mask(v, _mm512_set1_epi64((long long)x)));
}

__attribute__((target("avx512f"))) inline uint32_t count512_128(const uint64_t* kh, const uint64_t* kl, uint64_t xh,
                                                                uint64_t xl)
{
    const __m512i h = _mm512_load_si512(reinterpret_cast<const void*>(kh));
    const __m512i l = _mm512_load_si512(reinterpret_cast<const void*>(kl));
    const __m512i vh = _mm512_set1_epi64((long long)xh);
    const __mmask8 lt = _mm512_cmplt_epu64_mask(h, vh);
    const __mmask8 eq = _mm512_cmpeq_epu64_mask(h, vh);
    const __mmask8 le = _mm512_cmple_epu64_mask(l, _mm512_set1_epi64((long long)xl));
    return (uint32_t)__builtin_popcount((unsigned)(lt | (eq & le)));
}

// AVX2 has no unsigned 64-bit compare: flip the sign bits and compare signed.
__attribute__((target("avx2"))) inline __m256i flip(__m256i v)
{
    return _mm256_xor_si256(v, _mm256_set1_epi64x((long long)0x8000000000000000ull));
}

__attribute__((target("avx2"))) inline uint32_t mask4(__m256i v)
{
    return (uint32_t)_mm256_movemask_pd(_mm256_castsi256_pd(v));
}

__attribute__((target("avx2,popcnt"))) inline uint32_t count256_64(const uint64_t* k, uint64_t x)
{
    const __m256i vx = flip(_mm256_set1_epi64x((long long)x));
    uint32_t gt = 0;  // keys > x
    for (int h = 0; h < 2; ++h) {
        const __m256i v = flip(_mm256_load_si256(reinterpret_cast<const __m256i*>(k + 4 * h)));
        gt |= mask4(_mm256_cmpgt_epi64(v, vx)) << (4 * h);
    }
    return 8u - (uint32_t)__builtin_popcount(gt);
}

__attribute__((target("avx2,popcnt"))) inline uint32_t count256_128(const uint64_t* kh, const uint64_t* kl, uint64_t xh,
                                                                   uint64_t xl)
{
    const __m256i vh = flip(_mm256_set1_epi64x((long long)xh));
    const __m256i vl = flip(_mm256_set1_epi64x((long long)xl));
    uint32_t le = 0;
    for (int h = 0; h < 2; ++h) {
        const __m256i a = flip(_mm256_load_si256(reinterpret_cast<const __m256i*>(kh + 4 * h)));
        const __m256i b = flip(_mm256_load_si256(reinterpret_cast<const __m256i*>(kl + 4 * h)));
        const uint32_t lt = mask4(_mm256_cmpgt_epi64(vh, a));
        const uint32_t eq = mask4(_mm256_cmpeq_epi64(vh, a));
        const uint32_t lo_gt = mask4(_mm256_cmpgt_epi64(b, vl));
        le |= (lt | (eq & ~lo_gt & 0xFu)) << (4 * h);
    }
    return (uint32_t)__builtin_popcount(le);
}

// The count and the batch are inlined into range512 / range256, whose target
// attributes let the compiler inline the vector helpers there in turn.
template <Isa I, bool WIDE>
__attribute__((always_inline)) inline uint32_t count(const Tree& t, uint64_t node, uint64_t xh, uint64_t xl)
{
    const uint64_t* kh = t.hi.p + node * kKeys;
    if constexpr (I == Isa::avx512) {
        if constexpr (WIDE) return count512_128(kh, t.lo.p + node * kKeys, xh, xl);
        else return count512_64(kh, xh);
    } else {
        if constexpr (WIDE) return count256_128(kh, t.lo.p + node * kKeys, xh, xl);
        else return count256_64(kh, xh);
    }
}

// One batch of up to kBatch addresses through all D levels (unrolled).
template <Isa I, bool WIDE, int D>
__attribute__((always_inline)) inline void batch(const Tree& t, const planb_addr_t* a, uint16_t* out, int n)
{
    uint64_t xh[kBatch], xl[kBatch], q[kBatch];
    for (int i = 0; i < n; ++i) {
        xh[i] = a[i].hi;
        xl[i] = WIDE ? a[i].lo : 0;
        q[i] = 0;
    }
#pragma GCC unroll 16
    for (int l = 0; l + 1 < D; ++l) {
        const uint64_t off = t.off[l], nxt = t.off[l + 1], lim = t.last[l + 1];
        for (int i = 0; i < n; ++i) {
            q[i] = std::min<uint64_t>(q[i] * kFan + count<I, WIDE>(t, off + q[i], xh[i], xl[i]), lim);
            __builtin_prefetch(t.hi.p + (nxt + q[i]) * kKeys);
            if constexpr (WIDE) __builtin_prefetch(t.lo.p + (nxt + q[i]) * kKeys);
        }
    }
    const uint64_t leaf0 = t.off[D - 1];
    for (int i = 0; i < n; ++i) {
        const uint32_t c = count<I, WIDE>(t, leaf0 + q[i], xh[i], xl[i]);  // >= 1: interval 0 starts at 0
        const uint64_t idx = std::min<uint64_t>(q[i] * kKeys + c - 1, t.m - 1);
        out[i] = t.nh[idx];
    }
}

template <bool WIDE, int D>
__attribute__((target("avx512f,popcnt"))) void range512(const Tree& t, const planb_addr_t* a, uint16_t* out, size_t lo,
                                                         size_t hi)
{
    for (size_t s = lo; s < hi; s += kBatch)
        batch<Isa::avx512, WIDE, D>(t, a + s, out + s, (int)std::min<size_t>(kBatch, hi - s));
}

template <bool WIDE, int D>
__attribute__((target("avx2,popcnt"))) void range256(const Tree& t, const planb_addr_t* a, uint16_t* out, size_t lo,
                                                      size_t hi)
{
    for (size_t s = lo; s < hi; s += kBatch)
        batch<Isa::avx2, WIDE, D>(t, a + s, out + s, (int)std::min<size_t>(kBatch, hi - s));
}

using RangeFn = void (*)(const Tree&, const planb_addr_t*, uint16_t*, size_t, size_t);

template <Isa I, bool WIDE, int D = 1>
RangeFn pick_depth(uint32_t depth)
{
    if constexpr (D > kMaxDepth) {
        return nullptr;
    } else {
        if (depth == (uint32_t)D) return I == Isa::avx512 ? range512<WIDE, D> : range256<WIDE, D>;
        return pick_depth<I, WIDE, D + 1>(depth);
    }
}

RangeFn pick(const Tree& t)
{
    const bool wide = t.key_bits == 128;
    if (t.isa == Isa::avx512) return wide ? pick_depth<Isa::avx512, true>(t.depth) : pick_depth<Isa::avx512, false>(t.depth);
    return wide ? pick_depth<Isa::avx2, true>(t.depth) : pick_depth<Isa::avx2, false>(t.depth);
}

Isa host_isa()
{
    __builtin_cpu_init();
    return __builtin_cpu_supports("avx512f") ? Isa::avx512 : Isa::avx2;
}

}  // namespace

extern "C" {

planb_cpu_tree_t* planb_cpu_tree_build(const planb_addr_t* starts, const uint16_t* next_hops, size_t m,
                                       uint32_t key_bits)
{
    if (!starts || !next_hops || m == 0 || (key_bits != 64 && key_bits != 128)) return nullptr;
    if (starts[0].hi != 0 || starts[0].lo != 0) return nullptr;
    for (size_t i = 0; i < m; ++i) {
        if (key_bits == 64 && starts[i].lo != 0) return nullptr;  // 64-bit keys would be inexact
        if (i && !(starts[i - 1].hi < starts[i].hi || (starts[i - 1].hi == starts[i].hi && starts[i - 1].lo < starts[i].lo)))
            return nullptr;  // not strictly increasing
    }
    auto* t = new (std::nothrow) planb_cpu_tree();
    if (!t) return nullptr;
    t->key_bits = key_bits;
    t->m = m;
    t->isa = host_isa();
    // smallest D with 8 * 9^(D-1) >= m
    uint64_t cap = kKeys;
    uint32_t D = 1;
    while (cap < m) {
        cap *= kFan;
        ++D;
    }
    if (D > (uint32_t)kMaxDepth) {
        delete t;
        return nullptr;
    }
    t->depth = D;
    const uint64_t leaves = (m + kKeys - 1) / kKeys;
    // nodes of level l: those covering an existing leaf; a node of level l spans 9^(D-1-l) leaves
    uint64_t nodes[kMaxDepth], total = 0;
    for (uint32_t l = 0; l < D; ++l) {
        uint64_t span = 1;
        for (uint32_t k = l + 1; k < D; ++k) span *= kFan;
        nodes[l] = (leaves + span - 1) / span;
        t->off[l] = total;
        t->last[l] = nodes[l] - 1;
        total += nodes[l];
    }
    if (!t->hi.alloc(total * kKeys) || (key_bits == 128 && !t->lo.alloc(total * kKeys))) {
        delete t;
        return nullptr;
    }
    auto put = [&](uint64_t node, int s, uint64_t key_index) {
        const bool real = key_index < m;
        t->hi.p[node * kKeys + s] = real ? starts[key_index].hi : ~0ull;
        if (key_bits == 128) t->lo.p[node * kKeys + s] = real ? starts[key_index].lo : ~0ull;
    };
    for (uint32_t l = 0; l < D; ++l) {
        uint64_t leafspan = 1;  // leaves under one child of a level-l node
        for (uint32_t k = l + 2; k < D; ++k) leafspan *= kFan;
        for (uint64_t q = 0; q < nodes[l]; ++q)
            for (int s = 0; s < kKeys; ++s) {
                if (l + 1 == D) {
                    put(t->off[l] + q, s, q * kKeys + (uint64_t)s);  // leaf: the starts in order
                } else {
                    // separator s: the minimum of child s + 1's subtree, i.e. the
                    // first key of its first leaf (a sentinel past the end)
                    const uint64_t child = q * kFan + (uint64_t)s + 1;
                    put(t->off[l] + q, s, child * leafspan * kKeys);
                }
            }
    }
    t->nh.assign(next_hops, next_hops + m);
    return t;
}

void planb_cpu_tree_free(planb_cpu_tree_t* tree) { delete tree; }

const char* planb_cpu_tree_isa(const planb_cpu_tree_t* tree)
{
    if (!tree) return "";
    return tree->isa == Isa::avx512 ? "avx512" : "avx2";
}

int planb_cpu_tree_depth(const planb_cpu_tree_t* tree) { return tree ? (int)tree->depth : PLANB_EINVAL; }

int planb_cpu_tree_lookup(const planb_cpu_tree_t* tree, const planb_addr_t* addrs, size_t n, uint16_t* out,
                          int threads)
{
    if (!tree || (n && (!addrs || !out))) return PLANB_EINVAL;
    if (n == 0) return PLANB_OK;
    const RangeFn fn = pick(*tree);
    if (!fn) return PLANB_EINVAL;
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const unsigned T = threads > 0 ? (unsigned)threads : hw;
    const size_t chunk = ((n + T - 1) / T + kBatch - 1) / kBatch * kBatch;
    std::vector<std::thread> th;
    for (unsigned k = 1; k < T && k * chunk < n; ++k)
        th.emplace_back(fn, std::cref(*tree), addrs, out, k * chunk, std::min(n, (k + 1) * chunk));
    fn(*tree, addrs, out, 0, std::min(n, chunk));
    for (auto& x : th) x.join();
    return PLANB_OK;
}

}  // extern "C"
