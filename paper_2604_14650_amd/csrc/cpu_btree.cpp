// CPU linearized B+-tree lookup: the host-core baseline the GPU kernel is
// measured against.  It descends the same byte image planb_build uploads
// (planb_build_image), following the paper's CPU design (Section 3, Algorithm 1;
// "Batching" and "Branch-free Search"): every node is searched by counting the
// keys <= x over all its slots (no early exit, so the compiler vectorizes it),
// the child is chosen arithmetically, and a group of addresses descends level
// by level together so that their node fetches overlap (each next node is
// prefetched as soon as its index is known).  Threads split the batch.
//
// This is not called by any GPU entry point and is no fallback for them.
#include <algorithm>
#include <cstring>
#include <thread>
#include <vector>

#include "../../include/planb.h"
#include "leaf_format.hpp"

namespace {

constexpr int kGroup = 16;  // addresses descending together

struct Tree {
    const uint8_t* img;
    uint64_t leaf_base, m_minus_1;
    uint32_t depth;
    uint64_t off[PLANB_MAX_LEVELS];   // first node of each internal level
    uint64_t last[PLANB_MAX_LEVELS];  // last node of each level
};

// keys <= x among the first S slots at p (KB: 4 = top 32 bits, 8 = high
// words only, 16 = {hi, lo})
template <int KB, int S>
inline uint32_t count_keys(const uint8_t* p, uint64_t xh, uint64_t xl)
{
    uint32_t c = 0;
    if constexpr (KB == 4) {
        uint32_t k[S];
        std::memcpy(k, p, sizeof(k));
        const uint32_t x = (uint32_t)(xh >> 32);
        for (int s = 0; s < S; ++s) c += k[s] <= x;
    } else if constexpr (KB == 8) {
        uint64_t k[S];
        std::memcpy(k, p, sizeof(k));
        for (int s = 0; s < S; ++s) c += k[s] <= xh;
    } else {
        uint64_t k[2 * S];
        std::memcpy(k, p, sizeof(k));
        for (int s = 0; s < S; ++s) c += (k[2 * s] < xh) | ((k[2 * s] == xh) & (k[2 * s + 1] <= xl));
    }
    return c;
}

template <int KB, int B>
void lookup_range(const Tree& t, const planb_addr_t* a, uint16_t* out, size_t lo, size_t hi)
{
    constexpr int LS = planb::leaf_slots_for(B, KB), LC = planb::leaf_cap_for(B, KB);
    for (size_t g0 = lo; g0 < hi; g0 += kGroup) {
        const int G = (int)std::min<size_t>(kGroup, hi - g0);
        uint64_t xh[kGroup], xl[kGroup];
        uint64_t q[kGroup];
        for (int i = 0; i < G; ++i) {
            xh[i] = a[g0 + i].hi;
            xl[i] = a[g0 + i].lo;
            q[i] = 0;
        }
        for (uint32_t l = 0; l + 1 < t.depth; ++l) {
            const bool to_leaf = l + 2 >= t.depth;
            for (int i = 0; i < G; ++i) {
                const uint8_t* node = t.img + (t.off[l] + q[i]) * B * KB;
                q[i] = std::min<uint64_t>(q[i] * B + count_keys<KB, B>(node, xh[i], xl[i]), t.last[l + 1]);
                const uint8_t* nxt = to_leaf ? t.img + (t.leaf_base + q[i] * LS) * KB : t.img + (t.off[l + 1] + q[i]) * B * KB;
                __builtin_prefetch(nxt);
                if (to_leaf && LS * KB > 64) __builtin_prefetch(nxt + 64);
            }
        }
        for (int i = 0; i < G; ++i) {
            const uint8_t* leaf = t.img + (t.leaf_base + q[i] * LS) * KB;
            uint32_t c;
            if constexpr (KB == 4) {  // blocks of five keys and their next hops
                uint32_t k[LS];
                std::memcpy(k, leaf, sizeof(k));
                const uint32_t x = (uint32_t)(xh[i] >> 32);
                c = 0;
                for (int s = 0; s < LS; ++s) c += (s % 8 < 5) & (k[s] <= x);
            } else if constexpr (KB == 8) {  // blocks of three keys and their next hops
                uint64_t k[LS];
                std::memcpy(k, leaf, sizeof(k));
                c = 0;
                for (int s = 0; s < LS; ++s) c += (s % 4 < 3) & (k[s] <= xh[i]);
            } else {
                c = count_keys<KB, LC>(leaf, xh[i], xl[i]);
            }
            const uint64_t idx = std::min<uint64_t>(q[i] * LC + c - 1, t.m_minus_1);
            uint16_t hop;
            std::memcpy(&hop, leaf + planb::leaf_hop_byte((uint32_t)(idx - q[i] * LC), KB, LC), 2);
            out[g0 + i] = hop;
        }
    }
}

using RangeFn = void (*)(const Tree&, const planb_addr_t*, uint16_t*, size_t, size_t);

template <int KB>
RangeFn pick_b(uint32_t b)
{
    return b == 8 ? lookup_range<KB, 8> : b == 16 ? lookup_range<KB, 16> : b == 32 ? lookup_range<KB, 32> : nullptr;
}

}  // namespace

extern "C" int planb_cpu_lookup(const void* image, const planb_info_t* info, const planb_addr_t* addrs, size_t n,
                                uint16_t* out, int threads)
{
    if (!image || !info || (n && (!addrs || !out))) return PLANB_EINVAL;
    if ((info->key_bits != 32 && info->key_bits != 64 && info->key_bits != 128) || info->depth == 0 ||
        info->depth > PLANB_MAX_LEVELS ||
        (info->fanout != 8 && info->fanout != 16 && info->fanout != 32) || info->leaf_keys == 0 ||
        info->intervals == 0)
        return PLANB_EINVAL;
    const int kb = (int)info->key_bits / 8, b = (int)info->fanout;
    if (info->leaf_keys != (uint32_t)planb::leaf_cap_for(b, kb) || info->leaf_slots != (uint32_t)planb::leaf_slots_for(b, kb))
        return PLANB_EINVAL;
    const RangeFn fn = kb == 4 ? pick_b<4>(info->fanout) : kb == 8 ? pick_b<8>(info->fanout) : pick_b<16>(info->fanout);
    Tree t{};
    t.img = static_cast<const uint8_t*>(image);
    t.depth = info->depth;
    t.leaf_base = info->leaf_base;
    t.m_minus_1 = info->intervals - 1;
    for (uint32_t l = 0; l < t.depth; ++l) {
        t.off[l] = info->level_offset[l];
        t.last[l] = info->level_nodes[l] - 1;
    }
    if (n == 0) return PLANB_OK;
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const unsigned T = threads > 0 ? (unsigned)threads : hw;
    const size_t chunk = (n + T - 1) / T;
    std::vector<std::thread> th;
    for (unsigned k = 1; k < T && k * chunk < n; ++k)
        th.emplace_back(fn, std::cref(t), addrs, out, k * chunk, std::min(n, (k + 1) * chunk));
    fn(t, addrs, out, 0, std::min(n, chunk));
    for (auto& x : th) x.join();
    return PLANB_OK;
}
