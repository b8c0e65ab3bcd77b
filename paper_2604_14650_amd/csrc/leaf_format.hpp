// Byte format of a leaf node, shared by the host builder and the kernels.
//
// A leaf holds a run of consecutive interval starts and, beside them, the
// next hop of each of those intervals, so that a lookup reads its answer from
// the cache line that held its leaf.  A leaf spans max(B slots, 128 bytes).
//  * 64-bit key slots: the leaf is a sequence of 32-byte blocks, each holding
//    three keys (24 bytes) followed by their three uint16 next hops (and two
//    bytes of padding), so 3/4 of the slots are keys;
//  * 32-bit key slots: 32-byte blocks of five keys (20 bytes), their five
//    next hops and two bytes of padding, so 5/8 of the slots are keys;
//  * 128-bit key slots: the keys first, then their next hops, as many pairs
//    as fit (7 in 128 bytes).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace planb {

__host__ __device__ constexpr int leaf_slots_for(int B, int key_bytes)
{
    return B * key_bytes >= 128 ? B : 128 / key_bytes;
}

__host__ __device__ constexpr int leaf_cap_for(int B, int key_bytes)
{
    return key_bytes == 4   ? leaf_slots_for(B, key_bytes) / 8 * 5
           : key_bytes == 8 ? leaf_slots_for(B, key_bytes) / 4 * 3
                            : leaf_slots_for(B, key_bytes) * key_bytes / (key_bytes + 2);
}

// Slot (within the leaf) of the leaf's key s, s < leaf_cap.
__host__ __device__ constexpr uint32_t leaf_key_slot(uint32_t s, int key_bytes)
{
    return key_bytes == 4 ? s / 5 * 8 + s % 5 : key_bytes == 8 ? s / 3 * 4 + s % 3 : s;
}

// Whether a slot of the leaf holds a key (or padding above the last interval,
// a sentinel) rather than next hops.
__host__ __device__ constexpr bool leaf_slot_is_key(uint32_t slot, int key_bytes, int leaf_cap)
{
    return key_bytes == 4 ? slot % 8 < 5 : key_bytes == 8 ? slot % 4 < 3 : slot < (uint32_t)leaf_cap;
}

// Byte (within the leaf) of the next hop of the leaf's interval s.
__host__ __device__ constexpr uint32_t leaf_hop_byte(uint32_t s, int key_bytes, int leaf_cap)
{
    return key_bytes == 4   ? s / 5 * 32 + 20 + s % 5 * 2
           : key_bytes == 8 ? s / 3 * 32 + 24 + s % 3 * 2
                            : (uint32_t)(leaf_cap * key_bytes) + 2 * s;
}

}  // namespace planb
