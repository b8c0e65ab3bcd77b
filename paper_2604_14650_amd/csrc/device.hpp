// Device-side descriptors and small wavefront helpers shared by the lookup
// kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "leaf_format.hpp"

namespace planb {

constexpr int kDevMaxLevels = 16;

// A 16-byte address record {hi, lo} as a native vector (for streaming loads).
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

// Staging from device memory into LDS: item i (i < count) is read by
// load(i) and written by store(i, v), the workgroup's threads taking items
// tid, tid + nthreads, ...  Each thread issues U reads before their stores, so
// a round of U items costs one memory round trip: a plain strided copy loop
// waits for every read before the next, and with a few dozen items per
// thread that wait was a large part of a launch's fixed cost.  Indices past the end
// are clamped to the last item, so every read and store is unconditional (a
// conditional store let the compiler sink its read behind the others' wait);
// the last item is then written more than once, always with its own value.
template <int U, typename Load, typename Store>
__device__ inline void stage_items(uint32_t count, uint32_t tid, uint32_t nthreads, Load load, Store store)
{
    if (count == 0) return;
    for (uint32_t i = tid; i < count; i += (uint32_t)U * nthreads) {
        decltype(load(0u)) v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = load(min(i + (uint32_t)u * nthreads, count - 1));
#pragma unroll
        for (int u = 0; u < U; ++u) store(min(i + (uint32_t)u * nthreads, count - 1), v[u]);
    }
}

// What a kernel needs to descend one built tree.  Passed by value (kernarg).
struct TreeDesc {
    const void* keys;        // slot array: internal nodes of B slots, then leaves
    uint32_t key_bytes;      // 16: full 128-bit keys {hi, lo}; 8: the hi word only (every key's lo is 0)
    const uint16_t* vals;    // next hop of interval i at vals[i] (also stored in the leaves)
    uint64_t m_minus_1;      // last interval index
    uint32_t depth;          // D, levels including the leaf level
    uint32_t lds_levels;     // top levels staged in LDS (<= depth)
    uint32_t lds_slots;      // slots in those levels (a prefix of the slot array)
    uint32_t fanout;         // B (checked against the kernel's template)
    uint32_t leaf_base;      // slot of the first leaf
    uint32_t last_hop;       // next hop of the last interval (vals[m_minus_1])
    uint32_t off[kDevMaxLevels];   // first node of each internal level
    uint32_t last[kDevMaxLevels];  // last allocated node of each level (the leaf level last)
};

// Key formats by slot width KB.  16: the record {hi, lo}, compared as a
// 128-bit unsigned integer.  8: only hi is stored, which a tree uses when
// every key's lo word is zero; then key <= x exactly when key.hi <= x.hi.
// 4: only the top 32 bits are stored, when every key's low 96 bits are zero
// (every prefix at most /32, e.g. IPv4 rules placed in the top 32 bits);
// then key <= x exactly when those 32 bits of the key are <= x's.
template <int KB>
struct KeyFmt;

template <>
struct KeyFmt<16> {
    using T = uint4;
    static __device__ __forceinline__ int le(uint4 k, uint64_t xhi, uint64_t xlo)
    {
        const uint64_t khi = ((uint64_t)k.y << 32) | k.x;
        const uint64_t klo = ((uint64_t)k.w << 32) | k.z;
        return (khi < xhi) | ((khi == xhi) & (klo <= xlo));
    }
};

template <>
struct KeyFmt<8> {
    using T = uint64_t;
    static __device__ __forceinline__ int le(uint64_t k, uint64_t xhi, uint64_t) { return k <= xhi; }
};

template <>
struct KeyFmt<4> {
    using T = uint32_t;
    static __device__ __forceinline__ int le(uint32_t k, uint64_t xhi, uint64_t) { return k <= (uint32_t)(xhi >> 32); }
};

// Sum of v over aligned groups of G consecutive lanes; every lane of a group
// receives the group's total.  G <= 16 stays inside one DPP row.
template <int G>
__device__ __forceinline__ int group_sum(int v)
{
    // every source lane of these patterns lies inside the row, so bound_ctrl
    // (0 for an invalid source) never applies; it spares a zeroed old value
    if constexpr (G >= 2) v += __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);   // quad_perm 1,0,3,2
    if constexpr (G >= 4) v += __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);   // quad_perm 2,3,0,1
    if constexpr (G >= 8) v += __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true);  // row_half_mirror
    if constexpr (G >= 16) v += __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, true); // row_mirror
    if constexpr (G >= 32) v += __shfl_xor(v, 16, 64);
    return v;
}

}  // namespace planb
