// Learned-model descriptors shared by the learned kernels, the table set and
// the server.
#pragma once

#include "api_internal.hpp"
#include "multi.hpp"

namespace planb {

// What a kernel needs of one trained model (wb == nullptr: no model).
struct ModelDesc {
    const uint16_t* wb;  // bfloat16 copy of the flat parameter vector (W1, W2, w3 are read from it)
    const float* w;      // float32 master vector (biases are read from it)
    const uint32_t* eps; // per-segment error bound, kEmpty = no training point predicts there
    uint32_t segments;
    float seg_scale;      // segments / m for m intervals: a lookup's error-table segment is about p * seg_scale
};

// Device bytes a model with `segments` error-table entries holds (weights,
// their bf16 copy, Adam moments, error table, gradient partials), plus its
// leaf tops for a tree of `nleaves` leaves with 64-bit key slots (else 0).
size_t learned_model_bytes(uint32_t segments, uint64_t nleaves);

// The model of a FIB that has a trained model and error table, else all zero.
ModelDesc ready_model_desc(const planb_fib_t* f);

// Learned multi-FIB launch: per burst, the table's model and error table
// (or the tree descent where the table has no model).
int plan_multi_learned(int fanout, int kb, uint32_t max_bursts, MultiLaunch* L);
hipError_t launch_multi_learned(const MultiLaunch& L, const TreeDesc* tables, const ModelDesc* models,
                                uint32_t n_tables, const BurstRec* bursts, const uint32_t* count,
                                uint32_t max_bursts, uint32_t* fallbacks, hipStream_t stream);

}  // namespace planb
