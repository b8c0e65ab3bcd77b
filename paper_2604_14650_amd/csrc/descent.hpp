// One wavefront step of the batched tree descent, shared by the plain,
// multi-batch (persistent) and multi-FIB kernels.
//
// This is the search of the PlanB paper's Section 3 (Algorithm 1 and Listing 1)
// mapped onto a wave64: G = B / KPL lanes cooperate on one lookup.  Each lane
// compares KPL keys of the current node with the address x (strided by G so a
// group's loads are contiguous), the group adds its counts with DPP, and the
// count c of keys <= x selects child q*B + c.  At the leaf the interval index
// is q*(B-1) + c - 1.  Node indices are clamped to each level's last allocated
// node, which only alters the path of an address equal to the sentinel padding
// (all ones in the compared width); that address's answer is the last interval.
#pragma once

#include "device.hpp"

namespace planb {

template <int B, int KPL, int R, bool WIDE>
struct Descent {
    using KF = KeyFmt<WIDE>;
    using K = typename KF::T;
    static constexpr int G = B / KPL;                     // lanes per lookup
    static constexpr int LPW = 64 / G;                    // lookups per wavefront per step
    static constexpr uint64_t kStep = (uint64_t)LPW * R;  // lookups per wavefront step

    // Bytes of LDS the top levels of t take.
    static __host__ __device__ size_t lds_bytes(const TreeDesc& t) { return (size_t)t.lds_nodes * B * sizeof(K); }

    // Copy the first t.lds_nodes nodes (the top t.lds_levels levels) to LDS.
    static __device__ void stage(const TreeDesc& t, uint4* lds_raw, int tid, int nthreads)
    {
        const uint32_t units = t.lds_nodes * (uint32_t)(B * sizeof(K) / 16);
        const uint4* src = static_cast<const uint4*>(t.keys);
        for (uint32_t i = tid; i < units; i += nthreads) lds_raw[i] = src[i];
    }

    template <bool FROM_LDS>
    static __device__ __forceinline__ uint32_t node_count(const K* keys, size_t nb, uint64_t xhi, uint64_t xlo)
    {
        int cnt = 0;
#pragma unroll
        for (int s = 0; s < KPL; ++s) cnt += KF::le(keys[nb + s * G], xhi, xlo);
        return (uint32_t)group_sum<G>(cnt);
    }

    // Lookups [base, base + kStep) of a batch of n >= 1 addresses.  Every lane
    // of the wavefront must call this together (DPP crosses lanes).
    static __device__ __forceinline__ void step(const TreeDesc& t, const K* lds_keys, const u64x2* addrs,
                                                uint64_t base, uint64_t n, void* out, int index_out)
    {
        const int lane = threadIdx.x & 63;
        const int grp = lane / G;
        const int j = lane % G;
        const K* gkeys = static_cast<const K*>(t.keys);
        uint64_t xhi[R], xlo[R];
        uint32_t q[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t i = base + (uint64_t)r * LPW + grp;
            const u64x2 a = __builtin_nontemporal_load(addrs + (i < n ? i : n - 1));
            xhi[r] = a.x;
            xlo[r] = a.y;
            q[r] = 0;
        }
        for (uint32_t l = 0; l + 1 < t.depth; ++l) {
            const uint32_t off = t.off[l], lim = t.last[l + 1];
            if (l < t.lds_levels) {
#pragma unroll
                for (int r = 0; r < R; ++r)
                    q[r] = min(q[r] * B + node_count<true>(lds_keys, (size_t)(off + q[r]) * B + j, xhi[r], xlo[r]), lim);
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r)
                    q[r] = min(q[r] * B + node_count<false>(gkeys, (size_t)(off + q[r]) * B + j, xhi[r], xlo[r]), lim);
            }
        }
        const uint32_t loff = t.off[t.depth - 1];
        const bool leaf_lds = t.lds_levels >= t.depth;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const size_t nb = (size_t)(loff + q[r]) * B + j;
            const uint32_t c = leaf_lds ? node_count<true>(lds_keys, nb, xhi[r], xlo[r])
                                        : node_count<false>(gkeys, nb, xhi[r], xlo[r]);
            uint64_t idx = (uint64_t)q[r] * (B - 1) + c - 1;  // c >= 1: interval 0 starts at 0
            idx = idx < t.m_minus_1 ? idx : t.m_minus_1;
            const uint64_t i = base + (uint64_t)r * LPW + grp;
            if (j == 0 && i < n) {
                if (index_out)
                    __builtin_nontemporal_store((uint32_t)idx, static_cast<uint32_t*>(out) + i);
                else
                    __builtin_nontemporal_store(t.vals[idx], static_cast<uint16_t*>(out) + i);
            }
        }
    }
};

// Picks KernelOf<B, KPL, R, W, BS>::get() for runtime values among the
// compiled-in variants: B in {8, 16, 32}, KPL in {1, 2, 4, 8, 16} with B/KPL
// in [1, 32], R in {1, 2, 4}, W (wide keys) and BS in {512, 1024}.
template <template <int, int, int, bool, int> class KernelOf>
struct VariantTable {
    using Fn = typename KernelOf<8, 1, 1, true, 512>::Fn;

    template <int B, int KPL, bool W, int BS>
    static Fn by_r(int R)
    {
        switch (R) {
        case 1: return KernelOf<B, KPL, 1, W, BS>::get();
        case 2: return KernelOf<B, KPL, 2, W, BS>::get();
        case 4: return KernelOf<B, KPL, 4, W, BS>::get();
        default: return nullptr;
        }
    }
    template <int B, bool W, int BS>
    static Fn by_kpl(int kpl, int R)
    {
        switch (kpl) {
        case 1: return by_r<B, 1, W, BS>(R);
        case 2: return by_r<B, 2, W, BS>(R);
        case 4: return by_r<B, 4, W, BS>(R);
        case 8: return by_r<B, 8, W, BS>(R);
        case 16: if constexpr (B >= 16) return by_r<B, 16, W, BS>(R); else return nullptr;
        default: return nullptr;
        }
    }
    template <bool W, int BS>
    static Fn by_b(int B, int kpl, int R)
    {
        switch (B) {
        case 8: return by_kpl<8, W, BS>(kpl, R);
        case 16: return by_kpl<16, W, BS>(kpl, R);
        case 32: return by_kpl<32, W, BS>(kpl, R);
        default: return nullptr;
        }
    }
    static Fn pick(int B, int kpl, int R, bool wide, int bs)
    {
        if (bs == 512) return wide ? by_b<true, 512>(B, kpl, R) : by_b<false, 512>(B, kpl, R);
        if (bs == 1024) return wide ? by_b<true, 1024>(B, kpl, R) : by_b<false, 1024>(B, kpl, R);
        return nullptr;
    }
};

}  // namespace planb
