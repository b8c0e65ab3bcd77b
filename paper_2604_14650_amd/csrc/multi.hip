// Multi-FIB lookups: one persistent launch serves bursts that each name their
// own table (the paper's router serves one FIB per LPM thread; a serving GPU
// keeps many tables resident, e.g. one per VRF).  Tables are described by a
// device array of tree descriptors; bursts are cut into wavefront tiles like
// the uneven-batch kernel, and every tile descends its burst's table with all
// levels read through the caches (no per-table LDS staging).
#include "api_internal.hpp"
#include "burst_tiles.hpp"
#include "descent.hpp"
#include "learned.hpp"
#include "multi.hpp"

namespace planb {

template <int B, int KPL, int R, int KB, int BS, bool BIN>
__global__ void __launch_bounds__(BS)
multi_kernel(const TreeDesc* __restrict__ tables, uint32_t n_tables, const BurstRec* __restrict__ bursts,
             const uint32_t* __restrict__ count, uint32_t max_bursts)
{
    using D = Descent<B, KPL, R, KB, BIN>;
    extern __shared__ uint32_t lds_u32[];
    uint32_t* tile_off = lds_u32;                 // max_bursts + 1
    uint32_t* part = tile_off + max_bursts + 1;   // BS
    auto live = [&](uint32_t tb) { return tb < n_tables && tables[tb].depth != 0; };
    const uint32_t nb = plan_burst_tiles<BS>(bursts, count, max_bursts, D::kStep, live, tile_off, part);
    const uint32_t total = tile_off[nb];
    const uint32_t nwaves = gridDim.x * (BS / 64);
    for (uint32_t tile = blockIdx.x * (BS / 64) + (threadIdx.x >> 6); tile < total; tile += nwaves) {
        const uint32_t k = burst_of_tile(tile_off, nb, tile);
        const BurstRec br = bursts[k];
        const TreeDesc& t = tables[br.table];
        D::step(t, nullptr, br.addrs, (uint64_t)(tile - tile_off[k]) * D::kStep, br.n, br.out, 0);
    }
}

namespace {

template <int B, int KPL, int R, int KB, int BS, bool BIN>
struct MultiKernel {
    using Fn = void (*)(const TreeDesc*, uint32_t, const BurstRec*, const uint32_t*, uint32_t);
    static Fn get() { return multi_kernel<B, KPL, R, KB, BS, BIN>; }
};

}  // namespace

int plan_multi(int fanout, int kb, const LookupTuning& tu, uint32_t max_bursts, MultiLaunch* L)
{
    L->fn = reinterpret_cast<const void*>(VariantTable<MultiKernel>::pick(fanout, tu.kpl, tu.R, kb, tu.block, false));
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
    ModelDesc* dev_models = nullptr; // max_tables model descriptors (wb == NULL: no model)
    uint32_t max_tables = 0;
    int fanout = 0;                  // shared by every FIB of the set (0 until the first)
    int key_bytes = 0;
    int device = 0;
    LookupTuning tune;               // launch shape of the multi-FIB kernel
    UseLog uses;                     // streams with launches of this set
};

namespace {

// One event for the launch, shared by the set and by every FIB it names, so
// that a FIB freed later waits for this launch too.
void note_set_use(const planb_tableset_t* ts_c, hipStream_t stream)
{
    auto* ts = const_cast<planb_tableset_t*>(ts_c);
    UseRef ev = note_use(ts->uses, stream);
    for (const planb_fib_t* f : ts->fibs)
        if (f) note_shared_use(f->uses, stream, ev);
}

}  // namespace

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
    if (e == hipSuccess)
        e = fib_alloc(ts->device, reinterpret_cast<void**>(&ts->dev), sizeof(TreeDesc) * max_tables);
    if (e == hipSuccess) e = hipMemset(ts->dev, 0, sizeof(TreeDesc) * max_tables);
    if (e == hipSuccess)
        e = fib_alloc(ts->device, reinterpret_cast<void**>(&ts->dev_models), sizeof(ModelDesc) * max_tables);
    if (e == hipSuccess) e = hipMemset(ts->dev_models, 0, sizeof(ModelDesc) * max_tables);
    if (e != hipSuccess) {
        fail_hip(e, "creating a table set");
        free_after(ts->uses, ts->device, {ts->dev, ts->dev_models});
        delete ts;
        return nullptr;
    }
    return ts;
}

void planb_tableset_free(planb_tableset_t* ts)
{
    if (!ts) return;
    free_after(ts->uses, ts->device, {ts->dev, ts->dev_models});
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
    const ModelDesc md = ready_model_desc(fib);
    hipError_t e = hipSuccess;
    {  // launches of the set already enqueued read the descriptors when they run
        std::lock_guard<std::mutex> lk(ts->uses.mu);
        for (auto& u : ts->uses.last)
            if (e == hipSuccess && u.second && u.second->ev) e = hipEventSynchronize(u.second->ev);
    }
    if (e == hipSuccess) e = hipMemcpy(ts->dev + slot, &d, sizeof(TreeDesc), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ts->dev_models + slot, &md, sizeof(ModelDesc), hipMemcpyHostToDevice);
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
    int rc = plan_multi(ts->fanout, ts->key_bytes ? ts->key_bytes : 16, ts->tune, max_bursts, &L);
    if (rc != PLANB_OK) return rc;
    hipError_t e = launch_multi(L, ts->dev, ts->max_tables, reinterpret_cast<const BurstRec*>(bursts), n_bursts,
                                max_bursts, static_cast<hipStream_t>(stream));
    if (e == hipSuccess) note_set_use(ts, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? PLANB_OK : fail_hip(e, "multi-FIB launch");
}

int planb_lookup_multi_learned(const planb_tableset_t* ts, const planb_burst_t* bursts, const uint32_t* n_bursts,
                               uint32_t max_bursts, uint32_t* fallback_count, void* stream)
{
    if (!ts) return fail(PLANB_EINVAL, "NULL table set");
    if (max_bursts == 0 || ts->fanout == 0) return PLANB_OK;
    if (!bursts || !n_bursts || reinterpret_cast<uintptr_t>(bursts) % 8 ||
        reinterpret_cast<uintptr_t>(n_bursts) % 4 || reinterpret_cast<uintptr_t>(fallback_count) % 4)
        return fail(PLANB_EINVAL, "NULL or misaligned descriptor pointer");
    MultiLaunch L;
    int rc = plan_multi_learned(ts->fanout, ts->key_bytes ? ts->key_bytes : 16, max_bursts, &L);
    if (rc != PLANB_OK) return rc;
    hipError_t e = launch_multi_learned(L, ts->dev, ts->dev_models, ts->max_tables,
                                        reinterpret_cast<const BurstRec*>(bursts), n_bursts, max_bursts,
                                        fallback_count, static_cast<hipStream_t>(stream));
    if (e == hipSuccess) note_set_use(ts, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? PLANB_OK : fail_hip(e, "learned multi-FIB launch");
}

}  // extern "C"

namespace planb {
const TreeDesc* tableset_device(const planb_tableset_t* ts) { return ts->dev; }
const ModelDesc* tableset_models(const planb_tableset_t* ts) { return ts->dev_models; }
int tableset_plan_learned(const planb_tableset_t* ts, uint32_t max_bursts, MultiLaunch* L)
{
    return plan_multi_learned(ts->fanout ? ts->fanout : 16, ts->key_bytes ? ts->key_bytes : 16, max_bursts, L);
}
uint32_t tableset_capacity(const planb_tableset_t* ts) { return ts->max_tables; }
int tableset_plan(const planb_tableset_t* ts, uint32_t max_bursts, MultiLaunch* L)
{
    return plan_multi(ts->fanout ? ts->fanout : 16, ts->key_bytes ? ts->key_bytes : 16, ts->tune, max_bursts, L);
}
}  // namespace planb
