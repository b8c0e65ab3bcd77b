// Batched lookup kernels: descent of the linearized B+-tree (Algorithm 1 and
// Listing 1 of the PlanB paper, Section 3) for gfx950.
//
// Mapping of the paper's CPU design onto a wave64 GPU:
//  * the in-node SIMD compare (broadcast x, load the node's keys, one compare
//    per key, popcount of the mask) becomes G = B / KPL lanes that each load
//    KPL 16-byte keys of the node with coalesced loads, compare them with x as
//    128-bit unsigned integers, and add their counts with DPP row operations;
//  * batching becomes the grid: every lane group descends R independent
//    lookups at once, and each wavefront serves 64/G groups;
//  * "branch-free": the child index is arithmetic on the count, and every lane
//    executes the same D levels (the fixed search depth of the paper);
//  * the cache residency of the top levels becomes an LDS copy of the first
//    lds_levels levels made once per workgroup.
// The count c of keys <= x (an upper bound, as Listing 1's "x >= key" count)
// selects child q*B + c; at the leaf, interval index = q*(B-1) + c - 1.  Every
// per-level node index is clamped to the level's last allocated node, which
// only changes the path of x = 2^128 - 1 (equal to the sentinel padding), whose
// answer is the last interval.
#include "device.hpp"
#include "lookup.hpp"

#include <map>
#include <mutex>
#include <tuple>
#include <unordered_map>

namespace planb {

template <int B, int KPL, int R, bool WIDE, int BS>
__global__ void __launch_bounds__(BS)
lookup_kernel(TreeDesc t, const uint4* __restrict__ addrs, uint64_t n, void* __restrict__ out, int index_out)
{
    using KF = KeyFmt<WIDE>;
    using K = typename KF::T;
    constexpr int G = B / KPL;    // lanes per lookup
    constexpr int LPW = 64 / G;   // lookups per wavefront per step
    extern __shared__ uint4 lds_raw[];
    const K* lds_keys = reinterpret_cast<const K*>(lds_raw);
    const K* gkeys = static_cast<const K*>(t.keys);

    // stage the top levels (the first lds_nodes nodes of the array) in 16-byte units
    const uint32_t units = t.lds_nodes * (uint32_t)(B * sizeof(K) / 16);
    const uint4* src = static_cast<const uint4*>(t.keys);
    for (uint32_t i = threadIdx.x; i < units; i += BS) lds_raw[i] = src[i];
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int grp = lane / G;
    const int j = lane % G;
    const uint64_t wave = (uint64_t)blockIdx.x * (BS / 64) + (threadIdx.x >> 6);
    const uint64_t nwaves = (uint64_t)gridDim.x * (BS / 64);
    constexpr uint64_t per_step = (uint64_t)LPW * R;

    for (uint64_t base = wave * per_step; base < n; base += nwaves * per_step) {
        uint64_t xhi[R], xlo[R];
        uint32_t q[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t i = base + (uint64_t)r * LPW + grp;
            const u64x2 a = __builtin_nontemporal_load(reinterpret_cast<const u64x2*>(addrs) + (i < n ? i : n - 1));
            xhi[r] = a.x;
            xlo[r] = a.y;
            q[r] = 0;
        }
        // internal levels: count keys <= x, step to child q*B + count
        for (uint32_t l = 0; l + 1 < t.depth; ++l) {
            const uint32_t off = t.off[l], lim = t.last[l + 1];
            if (l < t.lds_levels) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const size_t nb = (size_t)(off + q[r]) * B + j;
                    int cnt = 0;
#pragma unroll
                    for (int s = 0; s < KPL; ++s) cnt += KF::le(lds_keys[nb + s * G], xhi[r], xlo[r]);
                    const uint32_t c = (uint32_t)group_sum<G>(cnt);
                    q[r] = min(q[r] * B + c, lim);
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const size_t nb = (size_t)(off + q[r]) * B + j;
                    int cnt = 0;
#pragma unroll
                    for (int s = 0; s < KPL; ++s) cnt += KF::le(gkeys[nb + s * G], xhi[r], xlo[r]);
                    const uint32_t c = (uint32_t)group_sum<G>(cnt);
                    q[r] = min(q[r] * B + c, lim);
                }
            }
        }
        // leaf level: count >= 1 always (interval 0 starts at address 0)
        const uint32_t loff = t.off[t.depth - 1];
        const bool leaf_lds = t.lds_levels >= t.depth;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const size_t nb = (size_t)(loff + q[r]) * B + j;
            int cnt = 0;
            if (leaf_lds) {
#pragma unroll
                for (int s = 0; s < KPL; ++s) cnt += KF::le(lds_keys[nb + s * G], xhi[r], xlo[r]);
            } else {
#pragma unroll
                for (int s = 0; s < KPL; ++s) cnt += KF::le(gkeys[nb + s * G], xhi[r], xlo[r]);
            }
            const uint32_t c = (uint32_t)group_sum<G>(cnt);
            uint64_t idx = (uint64_t)q[r] * (B - 1) + c - 1;
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
}

namespace {

using KernelFn = void (*)(TreeDesc, const uint4*, uint64_t, void*, int);

template <int B, int KPL, bool W, int BS>
KernelFn pick_r(int R)
{
    switch (R) {
    case 1: return lookup_kernel<B, KPL, 1, W, BS>;
    case 2: return lookup_kernel<B, KPL, 2, W, BS>;
    case 4: return lookup_kernel<B, KPL, 4, W, BS>;
    default: return nullptr;
    }
}

template <int B, bool W, int BS>
KernelFn pick_kpl(int kpl, int R)
{
    switch (kpl) {
    case 1: return pick_r<B, 1, W, BS>(R);
    case 2: return pick_r<B, 2, W, BS>(R);
    case 4: return pick_r<B, 4, W, BS>(R);
    case 8: return pick_r<B, 8, W, BS>(R);
    case 16: if constexpr (B >= 16) return pick_r<B, 16, W, BS>(R); else return nullptr;
    default: return nullptr;
    }
}

template <bool W, int BS>
KernelFn pick_b(int B, int kpl, int R)
{
    switch (B) {
    case 8: return pick_kpl<8, W, BS>(kpl, R);
    case 16: return pick_kpl<16, W, BS>(kpl, R);
    case 32: return pick_kpl<32, W, BS>(kpl, R);
    default: return nullptr;
    }
}

KernelFn pick(int B, int kpl, int R, bool wide, int bs)
{
    if (bs == 512) return wide ? pick_b<true, 512>(B, kpl, R) : pick_b<false, 512>(B, kpl, R);
    if (bs == 1024) return wide ? pick_b<true, 1024>(B, kpl, R) : pick_b<false, 1024>(B, kpl, R);
    return nullptr;
}

struct DevProps {
    int cus = 0;
    int max_lds = 0;
};

std::mutex g_mu;
std::unordered_map<int, DevProps> g_props;
std::map<std::tuple<uintptr_t, size_t, int>, int> g_blocks_per_cu;  // (kernel, lds bytes, device) -> blocks per CU

hipError_t dev_props(DevProps* p)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_props.find(dev);
    if (it != g_props.end()) {
        *p = it->second;
        return hipSuccess;
    }
    DevProps d;
    if ((e = hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&d.max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)) != hipSuccess)
        return e;
    g_props[dev] = d;
    *p = d;
    return hipSuccess;
}

hipError_t occupancy(KernelFn fn, int bs, size_t lds, int* blocks)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const auto key = std::make_tuple(reinterpret_cast<uintptr_t>(fn), lds, dev);
    {
        std::lock_guard<std::mutex> g(g_mu);
        auto it = g_blocks_per_cu.find(key);
        if (it != g_blocks_per_cu.end()) {
            *blocks = it->second;
            return hipSuccess;
        }
    }
    if (lds > 64 * 1024) {
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
        if (e != hipSuccess) return e;
    }
    int nb = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, bs, lds);
    if (e != hipSuccess) return e;
    if (nb < 1) nb = 1;
    std::lock_guard<std::mutex> g(g_mu);
    g_blocks_per_cu[key] = nb;
    *blocks = nb;
    return hipSuccess;
}

}  // namespace

bool lookup_variant_exists(int B, int kpl, int R, int bs) { return pick(B, kpl, R, true, bs) != nullptr; }

int max_lds_bytes()
{
    DevProps p;
    if (dev_props(&p) != hipSuccess) return 64 * 1024;
    return p.max_lds;
}

hipError_t launch_lookup(const TreeDesc& t, const LookupTuning& tu, const void* addrs, uint64_t n, void* out,
                         bool index_out, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    KernelFn fn = pick((int)t.fanout, tu.kpl, tu.R, t.key_bytes == 16, tu.block);
    if (!fn) return hipErrorInvalidValue;
    DevProps p;
    hipError_t e = dev_props(&p);
    if (e != hipSuccess) return e;
    const size_t lds = (size_t)t.lds_nodes * t.fanout * t.key_bytes;
    if (lds > (size_t)p.max_lds) return hipErrorInvalidValue;
    int nb = 1;
    if ((e = occupancy(fn, tu.block, lds, &nb)) != hipSuccess) return e;
    const int G = (int)t.fanout / tu.kpl;
    const uint64_t per_block = (uint64_t)(tu.block / 64) * (64 / G) * tu.R;
    const uint64_t want = (n + per_block - 1) / per_block;
    const uint64_t cap = (uint64_t)p.cus * nb;
    const unsigned grid = (unsigned)(want < cap ? want : cap);
    hipLaunchKernelGGL(fn, dim3(grid), dim3(tu.block), lds, stream, t, static_cast<const uint4*>(addrs), n, out,
                       index_out ? 1 : 0);
    return hipGetLastError();
}

}  // namespace planb
