// Cutting a launch's bursts into wavefront tiles: shared by the multi-FIB
// kernels.  Every workgroup computes, in LDS, the first tile of each burst
// (an exclusive prefix sum of tile counts), then its wavefronts take tiles in
// a grid stride and find each tile's burst by binary search.
#pragma once

#include "device.hpp"
#include "multi.hpp"

namespace planb {

// tile_off: max_bursts + 1 entries, part: BS entries (both LDS).  Tiles of
// bursts naming an empty or unknown table slot are not counted.  Returns the
// number of bursts nb; tile_off[nb] is the tile total.  Ends with a barrier.
template <int BS, typename Live>
__device__ uint32_t plan_burst_tiles(const BurstRec* bursts, const uint32_t* count, uint32_t max_bursts,
                                     uint64_t tile_lookups, Live live, uint32_t* tile_off, uint32_t* part)
{
    const uint32_t nb = min(*count, max_bursts);
    const uint32_t per = (nb + BS - 1) / BS;
    const uint32_t b0 = min(threadIdx.x * per, nb), b1 = min(b0 + per, nb);
    auto tiles_of = [&](uint32_t b) -> uint32_t {
        return live(bursts[b].table) ? (uint32_t)((bursts[b].n + tile_lookups - 1) / tile_lookups) : 0u;
    };
    uint32_t local = 0;
    for (uint32_t b = b0; b < b1; ++b) local += tiles_of(b);
    part[threadIdx.x] = local;
    __syncthreads();
    for (uint32_t o = 1; o < BS; o <<= 1) {
        uint32_t v = part[threadIdx.x];
        if (threadIdx.x >= o) v += part[threadIdx.x - o];
        __syncthreads();
        part[threadIdx.x] = v;
        __syncthreads();
    }
    uint32_t acc = part[threadIdx.x] - local;
    for (uint32_t b = b0; b < b1; ++b) {
        tile_off[b] = acc;
        acc += tiles_of(b);
    }
    if (threadIdx.x == BS - 1) tile_off[nb] = part[BS - 1];
    __syncthreads();
    return nb;
}

// The burst holding tile `tile` (tile_off[lo] <= tile < tile_off[lo + 1]).
__device__ inline uint32_t burst_of_tile(const uint32_t* tile_off, uint32_t nb, uint32_t tile)
{
    uint32_t lo = 0, hi = nb;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (tile_off[mid] <= tile) lo = mid; else hi = mid;
    }
    return lo;
}

}  // namespace planb
