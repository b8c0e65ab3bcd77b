// Data-parallel primitives of the device-side build: prefix sums and a stable
// LSD radix sort of (key, value) pairs, written for gfx950 with 256-thread
// workgroups that each own a tile of 2048 consecutive items.
//
// Scan: every workgroup scans its tile in LDS (each thread sums its eight
// consecutive items, the workgroup scans those 256 sums, each thread then
// writes its items), records the tile's total, and a second pass adds the
// scanned tile totals (themselves scanned by the same routine, recursively).
//
// Sort: 4 bits per pass, least significant digit first.  A pass counts the
// digits of every tile (LDS counters), takes the exclusive prefix sum of the
// counts in digit-major order (digit d of tile b then starts at that sum), and
// scatters every item to its digit's start plus the number of items with the
// same digit before it in the tile, which a workgroup computes from per-thread
// digit counts scanned in digit-major order.  Items of one thread are
// consecutive and threads are in order, so equal digits keep their order: each
// pass is stable, hence the sort is.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

namespace planb {
namespace dsort {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr uint32_t kTile = kThreads * kItems;
constexpr int kBins = 16;

inline uint32_t tiles_of(uint32_t n) { return (n + kTile - 1) / kTile; }

// Exclusive scan of one value per thread over the workgroup (LDS, 256
// entries); returns the thread's exclusive prefix and the total in *sum.
template <typename T>
__device__ inline T block_exclusive(T v, T* lds, T* sum)
{
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int o = 1; o < kThreads; o <<= 1) {
        const T a = t >= o ? lds[t - o] : T(0);
        __syncthreads();
        lds[t] += a;
        __syncthreads();
    }
    const T incl = lds[t];
    *sum = lds[kThreads - 1];
    __syncthreads();
    return incl - v;
}

// Tile-local scan; tile totals to sums[blockIdx.x].
template <typename T>
__global__ void __launch_bounds__(kThreads) scan_tiles_kernel(const T* __restrict__ in, T* __restrict__ out, uint32_t n,
                                                               T* __restrict__ sums, int inclusive)
{
    __shared__ T lds[kThreads];
    const uint32_t base = blockIdx.x * kTile + threadIdx.x * kItems;
    T v[kItems];
    T local = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        v[k] = base + k < n ? in[base + k] : T(0);
        local += v[k];
    }
    T total;
    T run = block_exclusive(local, lds, &total);
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const T next = run + v[k];
        if (base + k < n) out[base + k] = inclusive ? next : run;
        run = next;
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) add_offsets_kernel(T* __restrict__ out, uint32_t n, const T* __restrict__ offs)
{
    const uint32_t base = blockIdx.x * kTile + threadIdx.x * kItems;
    const T o = offs[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kItems; ++k)
        if (base + k < n) out[base + k] += o;
}

// Device buffers allocated by the caller's allocator (alloc(&p, bytes)).
template <typename T, typename Alloc>
hipError_t scan(Alloc& alloc, const T* in, T* out, uint32_t n, bool inclusive, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const uint32_t tiles = tiles_of(n);
    T* sums = nullptr;
    hipError_t e = alloc(reinterpret_cast<void**>(&sums), (size_t)tiles * sizeof(T));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_tiles_kernel<T>, dim3(tiles), dim3(kThreads), 0, st, in, out, n, sums, inclusive ? 1 : 0);
    if ((e = hipGetLastError()) != hipSuccess || tiles == 1) return e;
    // the tiles' totals, scanned (exclusive) in place, are their offsets
    if ((e = scan<T>(alloc, sums, sums, tiles, false, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(add_offsets_kernel<T>, dim3(tiles), dim3(kThreads), 0, st, out, n, sums);
    return hipGetLastError();
}

template <typename K>
__device__ inline uint32_t digit(K k, int shift)
{
    return (uint32_t)((uint64_t)k >> shift) & (kBins - 1);
}

// counts[d * tiles + tile]: items of the tile with digit d.
template <typename K>
__global__ void __launch_bounds__(kThreads) count_kernel(const K* __restrict__ keys, uint32_t n, int shift, uint32_t tiles,
                                                          uint32_t* __restrict__ counts)
{
    __shared__ uint32_t c[kBins];
    if (threadIdx.x < kBins) c[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t base = blockIdx.x * kTile + threadIdx.x * kItems;
#pragma unroll
    for (int k = 0; k < kItems; ++k)
        if (base + k < n) atomicAdd(&c[digit(keys[base + k], shift)], 1u);
    __syncthreads();
    if (threadIdx.x < kBins) counts[threadIdx.x * tiles + blockIdx.x] = c[threadIdx.x];
}

// Stable scatter of one pass; starts[d * tiles + tile] is where digit d of the
// tile begins in the output (the exclusive scan of counts).
template <typename K, typename V>
__global__ void __launch_bounds__(kThreads) scatter_kernel(const K* __restrict__ kin, const V* __restrict__ vin,
                                                            K* __restrict__ kout, V* __restrict__ vout, uint32_t n,
                                                            int shift, uint32_t tiles,
                                                            const uint32_t* __restrict__ starts)
{
    __shared__ uint32_t cnt[kBins * kThreads];  // digit-major: cnt[d * 256 + thread]
    __shared__ uint32_t part[kThreads];
    const int t = threadIdx.x;
    const uint32_t base = blockIdx.x * kTile + t * kItems;
    K key[kItems];
    uint32_t dg[kItems], rank[kItems];
    uint32_t mine[kBins];
#pragma unroll
    for (int d = 0; d < kBins; ++d) mine[d] = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const bool in = base + k < n;
        key[k] = in ? kin[base + k] : K(0);
        dg[k] = in ? digit(key[k], shift) : 0u;
        rank[k] = 0;
#pragma unroll
        for (int d = 0; d < kBins; ++d) {
            const bool hit = in && dg[k] == (uint32_t)d;
            rank[k] = hit ? mine[d] : rank[k];
            mine[d] += hit ? 1u : 0u;
        }
    }
#pragma unroll
    for (int d = 0; d < kBins; ++d) cnt[d * kThreads + t] = mine[d];
    __syncthreads();
    // exclusive scan of cnt in digit-major order: thread t owns entries [16t, 16t + 16)
    uint32_t own[kBins], s = 0;
#pragma unroll
    for (int j = 0; j < kBins; ++j) {
        own[j] = cnt[t * kBins + j];
        s += own[j];
    }
    uint32_t total;
    uint32_t run = block_exclusive(s, part, &total);
#pragma unroll
    for (int j = 0; j < kBins; ++j) {
        const uint32_t v = own[j];
        cnt[t * kBins + j] = run;
        run += v;
    }
    __syncthreads();
    // cnt[d * 256 + t] - cnt[d * 256] = items with digit d in threads before t
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        if (base + k >= n) continue;
        const uint32_t d = dg[k];
        const uint32_t pos = starts[d * tiles + blockIdx.x] + (cnt[d * kThreads + t] - cnt[d * kThreads]) + rank[k];
        kout[pos] = key[k];
        vout[pos] = vin[base + k];
    }
}

// Stable sort of (kin, vin) by the low `bits` bits of the keys into (kout,
// vout); the inputs are left unchanged.
template <typename K, typename V, typename Alloc>
hipError_t sort_pairs(Alloc& alloc, const K* kin, K* kout, const V* vin, V* vout, uint32_t n, unsigned bits,
                      hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const uint32_t tiles = tiles_of(n);
    const int passes = (int)((bits + 3) / 4);
    K* ktmp = nullptr;
    V* vtmp = nullptr;
    uint32_t* counts = nullptr;
    hipError_t e;
    if ((e = alloc(reinterpret_cast<void**>(&ktmp), (size_t)n * sizeof(K))) != hipSuccess ||
        (e = alloc(reinterpret_cast<void**>(&vtmp), (size_t)n * sizeof(V))) != hipSuccess ||
        (e = alloc(reinterpret_cast<void**>(&counts), (size_t)kBins * tiles * sizeof(uint32_t))) != hipSuccess)
        return e;
    const K* ks = kin;
    const V* vs = vin;
    for (int p = 0; p < passes; ++p) {
        // the last pass writes the output
        K* kd = ((passes - 1 - p) % 2 == 0) ? kout : ktmp;
        V* vd = ((passes - 1 - p) % 2 == 0) ? vout : vtmp;
        const int shift = 4 * p;
        hipLaunchKernelGGL(count_kernel<K>, dim3(tiles), dim3(kThreads), 0, st, ks, n, shift, tiles, counts);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = scan<uint32_t>(alloc, counts, counts, kBins * tiles, false, st)) != hipSuccess) return e;
        hipLaunchKernelGGL((scatter_kernel<K, V>), dim3(tiles), dim3(kThreads), 0, st, ks, vs, kd, vd, n, shift, tiles,
                           counts);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        ks = kd;
        vs = vd;
    }
    return hipSuccess;
}

}  // namespace dsort
}  // namespace planb
