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
#include "descent.hpp"
#include "lookup.hpp"

#include <map>
#include <mutex>
#include <tuple>
#include <unordered_map>

namespace planb {

template <int B, int KPL, int R, int KB, int BS, bool BIN>
__global__ void __launch_bounds__(BS)
lookup_kernel(TreeDesc t, const u64x2* __restrict__ addrs, uint64_t n, void* __restrict__ out, int index_out)
{
    using D = Descent<B, KPL, R, KB, BIN>;
    extern __shared__ uint4 lds_raw[];
    D::stage(t, lds_raw, threadIdx.x, BS);
    __syncthreads();
    const uint64_t wave = (uint64_t)blockIdx.x * (BS / 64) + (threadIdx.x >> 6);
    const uint64_t nwaves = (uint64_t)gridDim.x * (BS / 64);
    const auto* lds_keys = reinterpret_cast<const typename D::K*>(lds_raw);
    for (uint64_t base = wave * D::kStep; base < n; base += nwaves * D::kStep)
        D::step(t, lds_keys, addrs, base, n, out, index_out);
}

// The same over 4-byte IPv4 addresses (each standing for the 128-bit address
// with those 32 bits on top), for trees with 32-bit key slots.
template <int B, int KPL, int R, int KB, int BS, bool BIN>
__global__ void __launch_bounds__(BS)
lookup_v4_kernel(TreeDesc t, const uint32_t* __restrict__ addrs, uint64_t n, void* __restrict__ out, int index_out)
{
    using D = Descent<B, KPL, R, KB, BIN>;
    extern __shared__ uint4 lds_raw[];
    D::stage(t, lds_raw, threadIdx.x, BS);
    __syncthreads();
    const uint64_t wave = (uint64_t)blockIdx.x * (BS / 64) + (threadIdx.x >> 6);
    const uint64_t nwaves = (uint64_t)gridDim.x * (BS / 64);
    const auto* lds_keys = reinterpret_cast<const typename D::K*>(lds_raw);
    for (uint64_t base = wave * D::kStep; base < n; base += nwaves * D::kStep)
        D::step(t, lds_keys, addrs, base, n, out, index_out);
}

// Hybrid descent with the bottom internal level in LDS too, as the top 32
// bits of its 64- or 128-bit keys (a quarter or half of the bytes: for trees
// like the 200k-prefix backbone table that level then fits beside the exact
// levels above it, and a lookup's only tree access outside the CU is its
// leaf, unless its address ties a key's top half; then its lane reads that
// whole key, from the first slot of the leaf the key starts).  Results are
// those of lookup_kernel.
template <int B, int KPL, int R, int KB, int BS>
__global__ void __launch_bounds__(BS)
lookup_tops_kernel(TreeDesc t, const u64x2* __restrict__ addrs, uint64_t n, void* __restrict__ out, int index_out)
{
    using D = Descent<B, KPL, R, KB, true>;
    extern __shared__ uint4 lds_raw[];
    D::stage_bottom_tops(t, lds_raw, threadIdx.x, BS);
    __syncthreads();
    const uint64_t wave = (uint64_t)blockIdx.x * (BS / 64) + (threadIdx.x >> 6);
    const uint64_t nwaves = (uint64_t)gridDim.x * (BS / 64);
    for (uint64_t base = wave * D::kStep; base < n; base += nwaves * D::kStep)
        D::template step_hybrid<u64x2, true>(t, lds_raw, addrs, base, n, out, index_out);
}

// Binary search over the sorted interval starts, one lane per address: the
// GPU analogue of the paper's std::lower_bound baseline (Section 4's
// ablation), kept as the first rung of the design ladder.  Every probe is a
// dependent read of one key (about log2(m) of them), then one read of the
// next-hop array.  Keys are read in place from the leaves.
template <int B, int KB>
__global__ void __launch_bounds__(256)
bsearch_kernel(TreeDesc t, const u64x2* __restrict__ addrs, uint64_t n, uint16_t* __restrict__ out)
{
    using KF = KeyFmt<KB>;
    const uint64_t m = t.m_minus_1 + 1;
    uint64_t top = 1;
    while (top * 2 <= m) top *= 2;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const u64x2 a = __builtin_nontemporal_load(addrs + i);
        uint64_t c = 0;  // starts <= x (starts[0] = 0 <= x, so c >= 1)
        for (uint64_t step = top; step >= 1; step >>= 1) {
            const uint64_t probe = c + step - 1;
            if (probe < m && KF::le(leaf_key<B, KB>(t, probe), a.x, a.y)) c += step;
        }
        __builtin_nontemporal_store(t.vals[c - 1], out + i);
    }
}

namespace {

template <int B, int KPL, int R, int KB, int BS, bool BIN>
struct PlainKernel {
    using Fn = void (*)(TreeDesc, const u64x2*, uint64_t, void*, int);
    static Fn get() { return lookup_kernel<B, KPL, R, KB, BS, BIN>; }
};

using KernelFn = PlainKernel<8, 1, 1, 16, 512, false>::Fn;

template <int B, int KPL, int R, int KB, int BS, bool BIN>
struct V4Kernel {  // instantiated for 32-bit key slots only
    using Fn = void (*)(TreeDesc, const uint32_t*, uint64_t, void*, int);
    static Fn get()
    {
        if constexpr (KB == 4)
            return lookup_v4_kernel<B, KPL, R, KB, BS, BIN>;
        else
            return nullptr;
    }
};

KernelFn pick(int B, int kpl, int R, int kb, int bs, bool bin)
{
    return VariantTable<PlainKernel>::pick(B, kpl, R, kb, bs, bin);
}

// Key-tops kernels: B in {8, 16, 32}, B / KPL in {2, 4}, R in {1, 2, 4}, KB in {8, 16}, BS in {512, 1024}.
template <int B, int KPL, int KB>
KernelFn pick_tops_r(int R, int bs)
{
    auto by_bs = [&](auto r) -> KernelFn {
        constexpr int Rc = decltype(r)::value;
        return bs == 512    ? lookup_tops_kernel<B, KPL, Rc, KB, 512>
               : bs == 1024 ? lookup_tops_kernel<B, KPL, Rc, KB, 1024>
                            : nullptr;
    };
    return R == 1 ? by_bs(std::integral_constant<int, 1>{}) : R == 2 ? by_bs(std::integral_constant<int, 2>{})
         : R == 4 ? by_bs(std::integral_constant<int, 4>{}) : nullptr;
}

template <int KB>
KernelFn pick_tops_kb(int B, int kpl, int R, int bs)
{
    if (kpl <= 0 || B % kpl) return nullptr;
    const int G = B / kpl;
    if (B == 8) return G == 2 ? pick_tops_r<8, 4, KB>(R, bs) : G == 4 ? pick_tops_r<8, 2, KB>(R, bs) : nullptr;
    if (B == 16) return G == 2 ? pick_tops_r<16, 8, KB>(R, bs) : G == 4 ? pick_tops_r<16, 4, KB>(R, bs) : nullptr;
    if (B == 32) return G == 2 ? pick_tops_r<32, 16, KB>(R, bs) : G == 4 ? pick_tops_r<32, 8, KB>(R, bs) : nullptr;
    return nullptr;
}

KernelFn pick_tops(int B, int kpl, int R, int kb, int bs)
{
    return kb == 8 ? pick_tops_kb<8>(B, kpl, R, bs) : kb == 16 ? pick_tops_kb<16>(B, kpl, R, bs) : nullptr;
}

std::mutex g_mu;
std::unordered_map<int, DevProps> g_props;
std::map<std::tuple<uintptr_t, size_t, int>, int> g_blocks_per_cu;  // (kernel, lds bytes, device) -> blocks per CU

}  // namespace

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

hipError_t occupancy(const void* fn, int bs, size_t lds, int* blocks)
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
        e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
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

bool lookup_variant_exists(int B, int kpl, int R, int bs, bool bin) { return pick(B, kpl, R, 16, bs, bin) != nullptr; }

bool lookup_tops_variant_exists(int B, int kpl, int R, int kb, int bs) { return pick_tops(B, kpl, R, kb, bs) != nullptr; }

int max_lds_bytes()
{
    DevProps p;
    if (dev_props(&p) != hipSuccess) return 64 * 1024;
    return p.max_lds;
}

hipError_t launch_bsearch(const TreeDesc& t, const void* addrs, uint64_t n, uint16_t* out, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    using Fn = void (*)(TreeDesc, const u64x2*, uint64_t, uint16_t*);
    auto by_kb = [&](auto b) -> Fn {
        constexpr int Bc = decltype(b)::value;
        return t.key_bytes == 4 ? bsearch_kernel<Bc, 4> : t.key_bytes == 8 ? bsearch_kernel<Bc, 8> : bsearch_kernel<Bc, 16>;
    };
    Fn fn = t.fanout == 8 ? by_kb(std::integral_constant<int, 8>{})
          : t.fanout == 16 ? by_kb(std::integral_constant<int, 16>{})
          : t.fanout == 32 ? by_kb(std::integral_constant<int, 32>{}) : nullptr;
    if (!fn) return hipErrorInvalidValue;
    DevProps p;
    hipError_t e = dev_props(&p);
    if (e != hipSuccess) return e;
    int nb = 1;
    if ((e = occupancy(reinterpret_cast<const void*>(fn), 256, 0, &nb)) != hipSuccess) return e;
    const uint64_t want = (n + 255) / 256, cap = (uint64_t)p.cus * nb;
    hipLaunchKernelGGL(fn, dim3((unsigned)(want < cap ? want : cap)), dim3(256), 0, stream, t,
                       static_cast<const u64x2*>(addrs), n, out);
    return hipGetLastError();
}

hipError_t launch_lookup_v4(const TreeDesc& t, const LookupTuning& tu, const uint32_t* addrs, uint64_t n, void* out,
                            bool index_out, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    if (t.key_bytes != 4) return hipErrorInvalidValue;
    V4Kernel<8, 1, 1, 4, 512, false>::Fn fn = VariantTable<V4Kernel>::pick((int)t.fanout, tu.kpl, tu.R, 4, tu.block, tu.bin);
    if (!fn) return hipErrorInvalidValue;
    DevProps p;
    hipError_t e = dev_props(&p);
    if (e != hipSuccess) return e;
    const size_t lds = (size_t)t.lds_slots * t.key_bytes;
    if (lds > (size_t)p.max_lds) return hipErrorInvalidValue;
    int nb = 1;
    if ((e = occupancy(reinterpret_cast<const void*>(fn), tu.block, lds, &nb)) != hipSuccess) return e;
    const uint64_t per_block = (uint64_t)(tu.block / 64) * lookups_per_wave_step((int)t.fanout, tu);
    const uint64_t want = (n + per_block - 1) / per_block;
    const uint64_t cap = (uint64_t)p.cus * nb;
    const unsigned grid = (unsigned)(want < cap ? want : cap);
    hipLaunchKernelGGL(fn, dim3(grid), dim3(tu.block), lds, stream, t, addrs, n, out, index_out ? 1 : 0);
    return hipGetLastError();
}

constexpr uint64_t kTopsMinLookups = 1ull << 20;

hipError_t launch_lookup(const TreeDesc& td, const LookupTuning& tu, const void* addrs, uint64_t n, void* out,
                         bool index_out, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    TreeDesc t = td;
    KernelFn fn = nullptr;
    size_t slot_bytes = t.key_bytes;
    size_t extra = 0;
    // Below about 2^20 lookups the larger LDS staging of the key tops (one
    // workgroup per CU loading up to 160 KB) costs more than it saves: such
    // batches take the whole-key hybrid descent of the same tuning.
    if (tu.tops && n >= kTopsMinLookups) {
        if (t.key_bytes != 8 && t.key_bytes != 16) return hipErrorInvalidValue;
        // exact levels above the bottom internal one, then that level's key tops
        t.lds_levels = t.depth >= 2 ? t.depth - 2 : 0;
        t.lds_slots = t.off[t.lds_levels] * t.fanout;
        if (t.depth >= 2) extra = (size_t)(t.off[t.depth - 1] - t.off[t.depth - 2]) * (t.fanout - 1) * 4;
        fn = pick_tops((int)t.fanout, tu.kpl, tu.R, (int)t.key_bytes, tu.block);
    } else {
        fn = pick((int)t.fanout, tu.kpl, tu.R, (int)t.key_bytes, tu.block, tu.bin);
    }
    if (!fn) return hipErrorInvalidValue;
    DevProps p;
    hipError_t e = dev_props(&p);
    if (e != hipSuccess) return e;
    const size_t lds = (size_t)t.lds_slots * slot_bytes + extra;
    if (lds > (size_t)p.max_lds) return hipErrorInvalidValue;
    int nb = 1;
    if ((e = occupancy(reinterpret_cast<const void*>(fn), tu.block, lds, &nb)) != hipSuccess) return e;
    const uint64_t per_block = (uint64_t)(tu.block / 64) * lookups_per_wave_step((int)t.fanout, tu);
    const uint64_t want = (n + per_block - 1) / per_block;
    const uint64_t cap = (uint64_t)p.cus * nb;
    const unsigned grid = (unsigned)(want < cap ? want : cap);
    hipLaunchKernelGGL(fn, dim3(grid), dim3(tu.block), lds, stream, t, static_cast<const u64x2*>(addrs), n, out,
                       index_out ? 1 : 0);
    return hipGetLastError();
}

}  // namespace planb
