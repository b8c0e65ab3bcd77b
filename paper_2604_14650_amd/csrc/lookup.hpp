// Host-side launchers of the lookup kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "device.hpp"

namespace planb {

// Launch shape of the plain lookup kernel.
struct LookupTuning {
    int kpl = 4;      // keys each lane compares per node (B / kpl lanes per lookup)
    int R = 2;        // lookups each lane group keeps in flight
    int block = 512;  // threads per workgroup
    bool bin = false; // one lane per lookup, binary search, in the LDS-staged levels
    bool tops = false; // the bottom internal level in LDS as 32-bit key tops (64- and 128-bit
                       // key slots, hybrid shapes); the multi-FIB and IPv4 paths run as bin
};

// Lookups one wavefront handles per step of the descent for this shape.
inline uint64_t lookups_per_wave_step(int B, const LookupTuning& tu)
{
    const bool hybrid = tu.bin && tu.kpl < B;
    return hybrid ? 64ull * tu.R : (uint64_t)(64 / (B / tu.kpl)) * tu.R;
}

// Whether a (fanout, keys per lane, lookups per group, block size) kernel is compiled in.
bool lookup_variant_exists(int B, int kpl, int R, int bs, bool bin = false);
// The same for the key-tops kernel (64- and 128-bit key slots, kb = 8 or 16).
bool lookup_tops_variant_exists(int B, int kpl, int R, int kb, int bs);

// Largest dynamic LDS allocation a workgroup may request on the current device.
int max_lds_bytes();

struct DevProps {
    int cus = 0;
    int max_lds = 0;
};

// Compute units and LDS limit of the current device (cached per device).
hipError_t dev_props(DevProps* p);

// Resident workgroups per CU for kernel `fn` with `bs` threads and `lds`
// bytes of dynamic LDS (cached); raises the kernel's LDS limit when needed.
hipError_t occupancy(const void* fn, int bs, size_t lds, int* blocks);

// Enqueue one plain lookup over n addresses on `stream`; out receives uint16
// next hops, or uint32 interval indices when index_out.
hipError_t launch_lookup(const TreeDesc& t, const LookupTuning& tu, const void* addrs, uint64_t n, void* out,
                         bool index_out, hipStream_t stream);
// The same over 4-byte IPv4 addresses, for trees with 32-bit key slots.
hipError_t launch_lookup_v4(const TreeDesc& t, const LookupTuning& tu, const uint32_t* addrs, uint64_t n, void* out,
                            bool index_out, hipStream_t stream);
// Binary search over the sorted starts, one lane per address (ablation baseline).
hipError_t launch_bsearch(const TreeDesc& t, const void* addrs, uint64_t n, uint16_t* out, hipStream_t stream);

}  // namespace planb
