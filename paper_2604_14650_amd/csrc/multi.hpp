// Multi-FIB lookup kernel: records and launch helpers shared with the server.
#pragma once

#include "api_internal.hpp"

namespace planb {

struct BurstRec {  // same layout as planb_burst_t
    uint32_t table;
    uint32_t n;
    const u64x2* addrs;
    void* out;
};
static_assert(sizeof(BurstRec) == 24, "planb_burst_t layout");

struct MultiLaunch {
    const void* fn = nullptr;
    unsigned grid = 0;
    int block = 512;
    size_t lds = 0;
};

int plan_multi(int fanout, int kb, const LookupTuning& tu, uint32_t max_bursts, MultiLaunch* L);
hipError_t launch_multi(const MultiLaunch& L, const TreeDesc* tables, uint32_t n_tables, const BurstRec* bursts,
                        const uint32_t* count, uint32_t max_bursts, hipStream_t stream);

const TreeDesc* tableset_device(const planb_tableset_t* ts);
struct ModelDesc;
const ModelDesc* tableset_models(const planb_tableset_t* ts);
int tableset_plan_learned(const planb_tableset_t* ts, uint32_t max_bursts, MultiLaunch* L);
uint32_t tableset_capacity(const planb_tableset_t* ts);
int tableset_plan(const planb_tableset_t* ts, uint32_t max_bursts, MultiLaunch* L);

}  // namespace planb
