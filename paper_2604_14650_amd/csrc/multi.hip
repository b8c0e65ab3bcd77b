// Multi-FIB lookups: one persistent launch serves bursts that each name their
// own table (the paper's router serves one FIB per LPM thread; a serving GPU
// keeps many tables resident, e.g. one per VRF).  Tables are described by a
// device array of tree descriptors; bursts are cut into wavefront tiles like
// the uneven-batch kernel, and every tile descends its burst's table with all
// levels read through the caches (no per-table LDS staging).
#include "api_internal.hpp"
#include "descent.hpp"
#include "multi.hpp"

namespace planb {

template <int B, int KPL, int R, bool WIDE, int BS, bool BIN>
__global__ void __launch_bounds__(BS)
multi_kernel(const TreeDesc* __restrict__ tables, uint32_t n_tables, const BurstRec* __restrict__ bursts,
             const uint32_t* __restrict__ count, uint32_t max_bursts)
{
    using D = Descent<B, KPL, R, WIDE, BIN>;
    extern __shared__ uint32_t lds_u32[];
    uint32_t* tile_off = lds_u32;                 // max_bursts + 1
    uint32_t* part = tile_off + max_bursts + 1;   // BS
    const uint32_t nb = min(*count, max_bursts);
    const uint32_t per = (nb + BS - 1) / BS;
    const uint32_t b0 = min(threadIdx.x * per, nb), b1 = min(b0 + per, nb);
    auto tiles_of = [&](uint32_t b) -> uint32_t {  // bursts naming an empty or unknown slot are skipped
        const uint32_t tb = bursts[b].table;
        return tb < n_tables && tables[tb].depth ? (uint32_t)((bursts[b].n + D::kStep - 1) / D::kStep) : 0u;
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

    const uint32_t total = tile_off[nb];
    const uint32_t nwaves = gridDim.x * (BS / 64);
    for (uint32_t tile = blockIdx.x * (BS / 64) + (threadIdx.x >> 6); tile < total; tile += nwaves) {
        uint32_t lo = 0, hi = nb;  // tile_off[lo] <= tile < tile_off[hi]
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (tile_off[mid] <= tile) lo = mid; else hi = mid;
        }
        const BurstRec br = bursts[lo];
        const TreeDesc& t = tables[br.table];
        D::step(t, nullptr, br.addrs, (uint64_t)(tile - tile_off[lo]) * D::kStep, br.n, br.out, 0);
    }
}

namespace {

template <int B, int KPL, int R, bool W, int BS, bool BIN>
struct MultiKernel {
    using Fn = void (*)(const TreeDesc*, uint32_t, const BurstRec*, const uint32_t*, uint32_t);
    static Fn get() { return multi_kernel<B, KPL, R, W, BS, BIN>; }
};

}  // namespace

int plan_multi(int fanout, bool wide, const LookupTuning& tu, uint32_t max_bursts, MultiLaunch* L)
{
    L->fn = reinterpret_cast<const void*>(VariantTable<MultiKernel>::pick(fanout, tu.kpl, tu.R, wide, tu.block, false));
    if (!L->fn) return fail(PLANB_EINVAL, "no multi-FIB kernel for this fanout / tuning");
    DevProps p;
    hipError_t e = dev_props(&p);
    if (e != hipSuccess) return fail_hip(e, "device properties");
    L->block = tu.block;
    L->lds = ((size_t)max_bursts + 1 + tu.block) * 4;
    if (L->lds > (size_t)p.max_lds) return fail(PLANB_ERANGE, "too many bursts per launch for the LDS");
    int nb = 1;
    if ((e = occupancy(L->fn, tu.block, L->lds, &nb)) != hipSuccess) return fail_hip(e, "occupancy");
    L->grid = (unsigned)(p.cus * nb);
    return PLANB_OK;
}

hipError_t launch_multi(const MultiLaunch& L, const TreeDesc* tables, uint32_t n_tables, const BurstRec* bursts,
                        const uint32_t* count, uint32_t max_bursts, hipStream_t stream)
{
    void* args[] = {&tables, &n_tables, &bursts, &count, &max_bursts};
    return hipLaunchKernel(L.fn, dim3(L.grid), dim3(L.block), args, L.lds, stream);
}

}  // namespace planb

using namespace planb;

struct planb_tableset {
    TreeDesc* dev = nullptr;         // max_tables descriptors (depth 0 = empty slot)
    std::vector<TreeDesc> host;
    std::vector<const planb_fib_t*> fibs;
    uint32_t max_tables = 0;
    int fanout = 0;                  // shared by every FIB of the set (0 until the first)
    int key_bytes = 0;
    int device = 0;
    LookupTuning tune;               // launch shape of the multi-FIB kernel
};

extern "C" {

planb_tableset_t* planb_tableset_create(uint32_t max_tables)
{
    clear_error();
    if (max_tables == 0 || max_tables > (1u << 20)) {
        fail(PLANB_EINVAL, "max_tables must be 1 .. 2^20");
        return nullptr;
    }
    auto* ts = new (std::nothrow) planb_tableset_t();
    if (!ts) {
        fail(PLANB_ENOMEM, "out of host memory");
        return nullptr;
    }
    ts->max_tables = max_tables;
    ts->host.assign(max_tables, TreeDesc{});
    ts->fibs.assign(max_tables, nullptr);
    ts->tune.kpl = 4;
    ts->tune.R = 2;
    ts->tune.block = 512;
    hipError_t e = hipGetDevice(&ts->device);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&ts->dev), sizeof(TreeDesc) * max_tables);
    if (e == hipSuccess) e = hipMemset(ts->dev, 0, sizeof(TreeDesc) * max_tables);
    if (e != hipSuccess) {
        fail_hip(e, "creating a table set");
        if (ts->dev) (void)hipFree(ts->dev);
        delete ts;
        return nullptr;
    }
    return ts;
}

void planb_tableset_free(planb_tableset_t* ts)
{
    if (!ts) return;
    (void)hipDeviceSynchronize();
    if (ts->dev) (void)hipFree(ts->dev);
    delete ts;
}

int planb_tableset_set(planb_tableset_t* ts, uint32_t slot, const planb_fib_t* fib)
{
    if (!ts) return fail(PLANB_EINVAL, "NULL table set");
    if (slot >= ts->max_tables) return fail(PLANB_ERANGE, "slot out of range");
    TreeDesc d{};
    if (fib) {
        if (fib->device != ts->device) return fail(PLANB_EINVAL, "FIB and table set live on different devices");
        bool others = false;
        for (uint32_t k = 0; k < ts->max_tables; ++k) others |= (k != slot && ts->fibs[k] != nullptr);
        if (others && ((int)fib->lay.b != ts->fanout || (int)fib->key_bytes_per_slot != ts->key_bytes))
            return fail(PLANB_EINVAL, "every FIB of a table set needs the same fanout and key width");
        if (!others) {
            ts->fanout = (int)fib->lay.b;
            ts->key_bytes = (int)fib->key_bytes_per_slot;
            if (ts->fanout % ts->tune.kpl) ts->tune.kpl = 1;
        }
        d = fib->desc;
        d.lds_levels = 0;
        d.lds_slots = 0;
    }
    hipError_t e = hipMemcpy(ts->dev + slot, &d, sizeof(TreeDesc), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail_hip(e, "writing a table descriptor");
    ts->host[slot] = d;
    ts->fibs[slot] = fib;
    return PLANB_OK;
}

int planb_tableset_set_tuning(planb_tableset_t* ts, uint32_t keys_per_lane, uint32_t lookups_per_group,
                              uint32_t block_threads)
{
    if (!ts) return fail(PLANB_EINVAL, "NULL table set");
    const int b = ts->fanout ? ts->fanout : 16;
    if (!lookup_variant_exists(b, (int)keys_per_lane, (int)lookups_per_group, (int)block_threads) ||
        b % (int)keys_per_lane)
        return fail(PLANB_EINVAL, "unsupported multi-FIB tuning");
    ts->tune.kpl = (int)keys_per_lane;
    ts->tune.R = (int)lookups_per_group;
    ts->tune.block = (int)block_threads;
    return PLANB_OK;
}

int planb_lookup_multi(const planb_tableset_t* ts, const planb_burst_t* bursts, const uint32_t* n_bursts,
                       uint32_t max_bursts, void* stream)
{
    if (!ts) return fail(PLANB_EINVAL, "NULL table set");
    if (max_bursts == 0 || ts->fanout == 0) return PLANB_OK;  // nothing to do / no table yet
    if (!bursts || !n_bursts || reinterpret_cast<uintptr_t>(bursts) % 8 ||
        reinterpret_cast<uintptr_t>(n_bursts) % 4)
        return fail(PLANB_EINVAL, "NULL or misaligned descriptor pointer");
    MultiLaunch L;
    int rc = plan_multi(ts->fanout, ts->key_bytes == 16, ts->tune, max_bursts, &L);
    if (rc != PLANB_OK) return rc;
    hipError_t e = launch_multi(L, ts->dev, ts->max_tables, reinterpret_cast<const BurstRec*>(bursts), n_bursts,
                                max_bursts, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? PLANB_OK : fail_hip(e, "multi-FIB launch");
}

}  // extern "C"

namespace planb {
const TreeDesc* tableset_device(const planb_tableset_t* ts) { return ts->dev; }
uint32_t tableset_capacity(const planb_tableset_t* ts) { return ts->max_tables; }
int tableset_plan(const planb_tableset_t* ts, uint32_t max_bursts, MultiLaunch* L)
{
    return plan_multi(ts->fanout ? ts->fanout : 16, ts->key_bytes == 16, ts->tune, max_bursts, L);
}
}  // namespace planb
