// Uneven lookup batches in one persistent launch, HIP-graph replay of that
// launch, and the lookup autotuner.
//
// The paper forms its batches from NIC receive bursts and keeps many lookups in
// flight per core (Section 3 "Batching", "Loop Unrolling").  Here a persistent
// grid (compute units x resident workgroups) stages the top tree levels in LDS
// once, then walks a list of batches of any sizes: the batches are cut into
// wavefront steps ("tiles"), each workgroup computes the tile prefix sums in
// LDS, and every wavefront takes tiles in a fixed stride, so a launch needs no
// counters, atomics or memsets and can be captured into a graph once and
// replayed with new batch descriptors.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "api_internal.hpp"
#include "descent.hpp"

namespace planb {

struct BatchRec {  // same layout as planb_batch_t
    const u64x2* addrs;
    void* out;
    uint64_t n;
};
static_assert(sizeof(BatchRec) == sizeof(planb_batch_t), "planb_batch_t layout");

// Bytes of LDS the staged tree takes: the first t.lds_slots slots, and with
// TOPS the bottom internal level's key tops after them (B - 1 per node).
template <int B, int KB, bool TOPS>
__host__ __device__ inline size_t staged_tree_bytes(const TreeDesc& t)
{
    size_t bytes = (size_t)t.lds_slots * KB;
    if (TOPS && t.depth >= 2) bytes += (size_t)(t.off[t.depth - 1] - t.off[t.depth - 2]) * (B - 1) * 4;
    return (bytes + 15) / 16 * 16;
}

// TOPS: the descriptor's lds_levels are depth - 2 and the bottom internal
// level is staged as key tops (64-bit key slots; see lookup_tops_kernel).
template <int B, int KPL, int R, int KB, int BS, bool BIN, bool TOPS = false>
__global__ void __launch_bounds__(BS)
batches_kernel(TreeDesc t, const BatchRec* __restrict__ batches, const uint32_t* __restrict__ count,
               uint32_t max_batches, int index_out)
{
    using D = Descent<B, KPL, R, KB, BIN>;
    extern __shared__ uint4 lds_raw[];
    uint32_t* tile_off = reinterpret_cast<uint32_t*>(lds_raw + staged_tree_bytes<B, KB, TOPS>(t) / 16);  // max_batches + 1
    uint32_t* part = tile_off + max_batches + 1;                                                        // BS

    const uint32_t nb = min(*count, max_batches);
    const uint32_t per = (nb + BS - 1) / BS;
    const uint32_t b0 = min(threadIdx.x * per, nb), b1 = min(b0 + per, nb);
    uint32_t local = 0;
    for (uint32_t b = b0; b < b1; ++b) local += (uint32_t)((batches[b].n + D::kStep - 1) / D::kStep);
    part[threadIdx.x] = local;
    __syncthreads();
    for (uint32_t o = 1; o < BS; o <<= 1) {  // inclusive scan of the per-thread tile counts
        uint32_t v = part[threadIdx.x];
        if (threadIdx.x >= o) v += part[threadIdx.x - o];
        __syncthreads();
        part[threadIdx.x] = v;
        __syncthreads();
    }
    uint32_t acc = part[threadIdx.x] - local;
    for (uint32_t b = b0; b < b1; ++b) {
        tile_off[b] = acc;
        acc += (uint32_t)((batches[b].n + D::kStep - 1) / D::kStep);
    }
    if (threadIdx.x == BS - 1) tile_off[nb] = part[BS - 1];
    __syncthreads();

    // The grid is sized for the device (and fixed inside a graph); a
    // workgroup that gets no tile of this launch skips the LDS staging, which
    // would otherwise dominate launches of a few small batches.
    const uint32_t total = tile_off[nb];
    if (blockIdx.x * (uint32_t)(BS / 64) >= total) return;
    if constexpr (TOPS)
        D::stage_bottom_tops(t, lds_raw, threadIdx.x, BS);
    else
        D::stage(t, lds_raw, threadIdx.x, BS);
    __syncthreads();

    const auto* lds_keys = reinterpret_cast<const typename D::K*>(lds_raw);
    const uint32_t nwaves = gridDim.x * (BS / 64);
    for (uint32_t tile = blockIdx.x * (BS / 64) + (threadIdx.x >> 6); tile < total; tile += nwaves) {
        uint32_t lo = 0, hi = nb;  // tile_off[lo] <= tile < tile_off[hi]
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (tile_off[mid] <= tile) lo = mid; else hi = mid;
        }
        const BatchRec br = batches[lo];
        if constexpr (TOPS)
            D::template step_hybrid<u64x2, true>(t, lds_raw, br.addrs, (uint64_t)(tile - tile_off[lo]) * D::kStep, br.n,
                                                 br.out, index_out);
        else
            D::step(t, lds_keys, br.addrs, (uint64_t)(tile - tile_off[lo]) * D::kStep, br.n, br.out, index_out);
    }
}

namespace {

template <int B, int KPL, int R, int KB, int BS, bool BIN>
struct BatchesKernel {
    using Fn = void (*)(TreeDesc, const BatchRec*, const uint32_t*, uint32_t, int);
    static Fn get() { return batches_kernel<B, KPL, R, KB, BS, BIN>; }
};

using BatchesFn = BatchesKernel<8, 1, 1, 8, 512, false>::Fn;

struct BatchesLaunch {
    BatchesFn fn = nullptr;
    TreeDesc desc{};  // the FIB's, or with the key-tops staging
    unsigned grid = 0;
    size_t lds = 0;
};

// Key-tops variants: B in {8, 16, 32}, B / KPL in {2, 4}, R in {1, 2, 4}, KB in {8, 16}, BS in {512, 1024}.
template <int B, int KPL, int KB>
BatchesFn pick_tops_r(int R, int bs)
{
    auto by_bs = [&](auto r) -> BatchesFn {
        constexpr int Rc = decltype(r)::value;
        return bs == 512    ? batches_kernel<B, KPL, Rc, KB, 512, true, true>
               : bs == 1024 ? batches_kernel<B, KPL, Rc, KB, 1024, true, true>
                            : nullptr;
    };
    return R == 1 ? by_bs(std::integral_constant<int, 1>{}) : R == 2 ? by_bs(std::integral_constant<int, 2>{})
         : R == 4 ? by_bs(std::integral_constant<int, 4>{}) : nullptr;
}

template <int KB>
BatchesFn pick_batches_tops_kb(int B, int kpl, int R, int bs)
{
    if (kpl <= 0 || B % kpl) return nullptr;
    const int G = B / kpl;
    if (B == 8) return G == 2 ? pick_tops_r<8, 4, KB>(R, bs) : G == 4 ? pick_tops_r<8, 2, KB>(R, bs) : nullptr;
    if (B == 16) return G == 2 ? pick_tops_r<16, 8, KB>(R, bs) : G == 4 ? pick_tops_r<16, 4, KB>(R, bs) : nullptr;
    if (B == 32) return G == 2 ? pick_tops_r<32, 16, KB>(R, bs) : G == 4 ? pick_tops_r<32, 8, KB>(R, bs) : nullptr;
    return nullptr;
}

BatchesFn pick_batches_tops(int B, int kpl, int R, int kb, int bs)
{
    return kb == 8 ? pick_batches_tops_kb<8>(B, kpl, R, bs) : kb == 16 ? pick_batches_tops_kb<16>(B, kpl, R, bs) : nullptr;
}

int plan_batches(const planb_fib_t* fib, uint32_t max_batches, BatchesLaunch* L)
{
    const LookupTuning& tu = fib->tune;
    DevProps p;
    hipError_t e = dev_props(&p);
    if (e != hipSuccess) return fail_hip(e, "device properties");
    const size_t table = ((size_t)max_batches + 1 + tu.block) * 4;  // tile offsets and the scan
    L->desc = fib->desc;
    L->fn = nullptr;
    if (tu.tops) {  // the key-tops staging when it fits beside the batch table, else whole keys
        TreeDesc t = fib->desc;
        t.lds_levels = t.depth >= 2 ? t.depth - 2 : 0;
        t.lds_slots = t.off[t.lds_levels] * t.fanout;
        size_t tree = (size_t)t.lds_slots * t.key_bytes;
        if (t.depth >= 2) tree += (size_t)(t.off[t.depth - 1] - t.off[t.depth - 2]) * (t.fanout - 1) * 4;
        tree = (tree + 15) / 16 * 16;
        if (tree + table <= (size_t)p.max_lds) {
            L->fn = pick_batches_tops((int)t.fanout, tu.kpl, tu.R, (int)t.key_bytes, tu.block);
            L->desc = t;
            L->lds = tree + table;
        }
    }
    const TreeDesc& t = L->desc;
    if (!L->fn) {
        L->fn = VariantTable<BatchesKernel>::pick((int)t.fanout, tu.kpl, tu.R, (int)t.key_bytes, tu.block, tu.bin);
        L->lds = ((size_t)t.lds_slots * t.key_bytes + 15) / 16 * 16 + table;
    }
    if (!L->fn) return fail(PLANB_EINVAL, "no batches kernel for this tuning");
    if (L->lds > (size_t)p.max_lds)
        return fail(PLANB_ERANGE, "LDS levels plus " + std::to_string(max_batches) +
                                      " batch offsets exceed the workgroup LDS limit; lower lds_levels or max_batches");
    int nb = 1;
    if ((e = occupancy(reinterpret_cast<const void*>(L->fn), tu.block, L->lds, &nb)) != hipSuccess)
        return fail_hip(e, "occupancy");
    L->grid = (unsigned)(p.cus * nb);
    return PLANB_OK;
}

// Times every compiled-in tuning of the FIB's fanout and key width on the
// first n sample addresses (one warm-up and reps timed calls each) and applies
// the fastest.  Small calls (below 2^16 lookups) also try shallower LDS
// staging, which costs them more than it saves.
int autotune_core(planb_fib_t* fib, const planb_addr_t* sample, size_t n, uint32_t reps, hipStream_t st,
                  planb_autotune_result_t* res)
{
    if (reps == 0) reps = 3;
    const int max_lds = max_lds_bytes();
    const uint32_t b = fib->lay.b;
    int deepest = 0;
    while (deepest < (int)fib->lay.depth &&
           fib->lay.prefix_slots(deepest + 1) * (size_t)fib->key_bytes_per_slot <= (size_t)max_lds)
        ++deepest;
    const int shallowest = n < (1u << 16) ? 0 : std::max(0, deepest - 2);
    std::vector<planb_tuning_t> cands;
    for (uint32_t kpl = 1; kpl <= b && kpl <= 16; kpl *= 2) {
        if (b / kpl > 32) continue;
        for (uint32_t bin = 0; bin <= ((kpl == b || b / kpl == 2 || b / kpl == 4) ? 1u : 0u); ++bin)
            for (uint32_t R : {1u, 2u, 4u})
                for (uint32_t bs : {512u, 1024u})
                    for (int lds = shallowest; lds <= deepest; ++lds)
                        cands.push_back(planb_tuning_t{kpl, lds, R, bs, bin});
        // the bottom internal level as key tops (64- and 128-bit key slots; skipped
        // by planb_set_tuning when the levels do not fit a workgroup's LDS)
        if ((fib->key_bytes_per_slot == 8 || fib->key_bytes_per_slot == 16) && (b / kpl == 2 || b / kpl == 4))
            for (uint32_t R : {1u, 2u, 4u})
                for (uint32_t bs : {512u, 1024u}) cands.push_back(planb_tuning_t{kpl, deepest, R, bs, 2u});
    }
    uint16_t* out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&out), n * sizeof(uint16_t));
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    planb_tuning_t saved{};
    planb_get_tuning(fib, &saved);
    planb_tuning_t best = saved;
    float best_ms = -1.f;
    uint32_t tried = 0;
    for (size_t c = 0; e == hipSuccess && c < cands.size(); ++c) {
        if (planb_set_tuning(fib, &cands[c]) != PLANB_OK) continue;
        if (planb_lookup(fib, sample, n, out, st) != PLANB_OK) continue;  // warm-up
        if ((e = hipEventRecord(e0, st)) != hipSuccess) break;
        for (uint32_t r = 0; r < reps; ++r) planb_lookup(fib, sample, n, out, st);
        if ((e = hipEventRecord(e1, st)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess) break;
        float ms = 0.f;
        if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
        ms /= (float)reps;
        ++tried;
        if (best_ms < 0.f || ms < best_ms) {
            best_ms = ms;
            best = cands[c];
        }
    }
    if (out) (void)hipFree(out);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    planb_set_tuning(fib, &best);
    clear_error();
    if (e != hipSuccess) return fail_hip(e, "autotune timing");
    if (best_ms < 0.f) return fail(PLANB_EDEVICE, "no candidate tuning could be timed");
    res->tuning = best;
    res->ms_per_call = best_ms;
    res->glps = (float)((double)n / (best_ms * 1e-3) / 1e9);
    res->candidates = tried;
    return PLANB_OK;
}

}  // namespace
}  // namespace planb

using namespace planb;

struct planb_graph {
    static constexpr int kSlots = 4;
    const planb_fib_t* fib = nullptr;
    uint32_t max_batches = 0;
    uint64_t step = 1;  // lookups per tile of the captured variant
    hipStream_t cap = nullptr;
    struct Slot {
        unsigned char* host = nullptr;  // pinned: [count u32, pad to 16][BatchRec x max_batches]
        unsigned char* dev = nullptr;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipEvent_t done = nullptr;
        bool used = false;
    } slot[kSlots];
    int next = 0;
};

static void graph_release(planb_graph_t* g)
{
    for (auto& s : g->slot) {
        if (s.done) (void)hipEventSynchronize(s.done), (void)hipEventDestroy(s.done);
        if (s.exec) (void)hipGraphExecDestroy(s.exec);
        if (s.graph) (void)hipGraphDestroy(s.graph);
        if (s.dev) (void)hipFree(s.dev);
        if (s.host) (void)hipHostFree(s.host);
    }
    if (g->cap) (void)hipStreamDestroy(g->cap);
    delete g;
}

extern "C" {

int planb_lookup_batches(const planb_fib_t* fib, const planb_batch_t* batches, const uint32_t* n_batches,
                         uint32_t max_batches, void* stream)
{
    if (!fib) return fail(PLANB_EINVAL, "NULL fib");
    if (max_batches == 0) return PLANB_OK;
    if (!batches || !n_batches) return fail(PLANB_EINVAL, "NULL descriptor pointer");
    if (reinterpret_cast<uintptr_t>(batches) % 8 || reinterpret_cast<uintptr_t>(n_batches) % 4)
        return fail(PLANB_EINVAL, "misaligned descriptor pointer");
    int rc = check_current_device(fib);
    if (rc != PLANB_OK) return rc;
    BatchesLaunch L;
    if ((rc = plan_batches(fib, max_batches, &L)) != PLANB_OK) return rc;
    hipLaunchKernelGGL(L.fn, dim3(L.grid), dim3(fib->tune.block), L.lds, static_cast<hipStream_t>(stream), L.desc,
                       reinterpret_cast<const BatchRec*>(batches), n_batches, max_batches, 0);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) note_use(fib->uses, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? PLANB_OK : fail_hip(e, "batches launch");
}

planb_graph_t* planb_graph_create(const planb_fib_t* fib, uint32_t max_batches)
{
    clear_error();
    if (!fib || max_batches == 0) {
        fail(PLANB_EINVAL, "need a FIB and max_batches >= 1");
        return nullptr;
    }
    if (check_current_device(fib) != PLANB_OK) return nullptr;
    BatchesLaunch L;
    if (plan_batches(fib, max_batches, &L) != PLANB_OK) return nullptr;
    auto* g = new (std::nothrow) planb_graph_t();
    if (!g) {
        fail(PLANB_ENOMEM, "out of host memory");
        return nullptr;
    }
    g->fib = fib;
    g->max_batches = max_batches;
    g->step = lookups_per_wave_step((int)fib->desc.fanout, fib->tune);
    const size_t bytes = 16 + (size_t)max_batches * sizeof(BatchRec);
    hipError_t e = hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking);
    for (int k = 0; e == hipSuccess && k < planb_graph::kSlots; ++k) {
        auto& s = g->slot[k];
        if ((e = hipHostMalloc(reinterpret_cast<void**>(&s.host), bytes, hipHostMallocDefault)) != hipSuccess) break;
        std::memset(s.host, 0, bytes);
        if ((e = hipMalloc(reinterpret_cast<void**>(&s.dev), bytes)) != hipSuccess) break;
        if ((e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming)) != hipSuccess) break;
        if ((e = hipStreamBeginCapture(g->cap, hipStreamCaptureModeRelaxed)) != hipSuccess) break;
        (void)hipMemcpyAsync(s.dev, s.host, bytes, hipMemcpyHostToDevice, g->cap);
        hipLaunchKernelGGL(L.fn, dim3(L.grid), dim3(fib->tune.block), L.lds, g->cap, L.desc,
                           reinterpret_cast<const BatchRec*>(s.dev + 16), reinterpret_cast<const uint32_t*>(s.dev),
                           max_batches, 0);
        hipError_t le = hipGetLastError();
        e = hipStreamEndCapture(g->cap, &s.graph);
        if (e == hipSuccess) e = le;
        if (e != hipSuccess) break;
        if ((e = hipGraphInstantiate(&s.exec, s.graph, nullptr, nullptr, 0)) != hipSuccess) break;
    }
    if (e != hipSuccess) {
        fail_hip(e, "creating the lookup graph");
        graph_release(g);
        return nullptr;
    }
    return g;
}

int planb_graph_launch(planb_graph_t* g, const planb_batch_t* batches, uint32_t n_batches, void* stream)
{
    if (!g) return fail(PLANB_EINVAL, "NULL graph");
    if (n_batches > g->max_batches) return fail(PLANB_ERANGE, "more batches than the graph was created for");
    if (n_batches > 0 && !batches) return fail(PLANB_EINVAL, "NULL batches");
    uint64_t tiles = 0;
    for (uint32_t b = 0; b < n_batches; ++b) {
        const planb_batch_t& x = batches[b];
        if (x.n && (!x.addrs || !x.out)) return fail(PLANB_EINVAL, "NULL pointer in batch " + std::to_string(b));
        if (reinterpret_cast<uintptr_t>(x.addrs) % 16 || reinterpret_cast<uintptr_t>(x.out) % 2)
            return fail(PLANB_EINVAL, "misaligned pointer in batch " + std::to_string(b));
        tiles += (x.n + g->step - 1) / g->step;
    }
    if (tiles >= (1ull << 32)) return fail(PLANB_ERANGE, "too many lookups in one launch");
    auto& s = g->slot[g->next];
    g->next = (g->next + 1) % planb_graph::kSlots;
    hipError_t e;
    if (s.used && (e = hipEventSynchronize(s.done)) != hipSuccess) return fail_hip(e, "waiting for a graph slot");
    std::memcpy(s.host, &n_batches, sizeof(uint32_t));
    if (n_batches) std::memcpy(s.host + 16, batches, (size_t)n_batches * sizeof(BatchRec));
    if ((e = hipGraphLaunch(s.exec, static_cast<hipStream_t>(stream))) != hipSuccess)
        return fail_hip(e, "hipGraphLaunch");
    if ((e = hipEventRecord(s.done, static_cast<hipStream_t>(stream))) != hipSuccess)
        return fail_hip(e, "hipEventRecord");
    s.used = true;
    note_use(g->fib->uses, static_cast<hipStream_t>(stream));
    return PLANB_OK;
}

void planb_graph_free(planb_graph_t* g)
{
    if (g) graph_release(g);
}

int planb_autotune(planb_fib_t* fib, const planb_addr_t* sample, size_t n, uint32_t reps, void* stream,
                   planb_autotune_result_t* res)
{
    if (!fib || !res) return fail(PLANB_EINVAL, "NULL argument");
    if (n == 0 || !sample || reinterpret_cast<uintptr_t>(sample) % 16)
        return fail(PLANB_EINVAL, "need a non-empty, 16-byte aligned device sample");
    int rc = check_current_device(fib);
    if (rc != PLANB_OK) return rc;
    return autotune_core(fib, sample, n, reps, static_cast<hipStream_t>(stream), res);
}

int planb_autotune_sizes(planb_fib_t* fib, const planb_addr_t* sample, size_t n, const uint64_t* sizes, uint32_t count,
                         uint32_t reps, void* stream, planb_autotune_result_t* results)
{
    if (!fib || !sizes || !results || count == 0) return fail(PLANB_EINVAL, "NULL argument or no sizes");
    if (!sample || reinterpret_cast<uintptr_t>(sample) % 16) return fail(PLANB_EINVAL, "need a 16-byte aligned device sample");
    for (uint32_t k = 0; k < count; ++k) {
        if (sizes[k] == 0 || sizes[k] > n) return fail(PLANB_EINVAL, "every size must be in 1..n (the sample's length)");
        if (k && sizes[k] <= sizes[k - 1]) return fail(PLANB_EINVAL, "sizes must be strictly ascending");
    }
    int rc = check_current_device(fib);
    if (rc != PLANB_OK) return rc;
    planb_tuning_t saved{};
    planb_get_tuning(fib, &saved);
    std::vector<planb_fib_t::SizeTuning> keep;
    keep.swap(fib->size_tunings);  // time every candidate as the FIB's own tuning
    std::vector<uint64_t> lo(count);
    std::vector<planb_tuning_t> tu(count);
    for (uint32_t k = 0; k < count && rc == PLANB_OK; ++k) {
        rc = autotune_core(fib, sample, sizes[k], reps, static_cast<hipStream_t>(stream), &results[k]);
        tu[k] = results[k].tuning;
        // bucket k serves calls from the geometric midpoint below its size
        lo[k] = k == 0 ? 1 : (uint64_t)std::ceil(std::sqrt((double)sizes[k - 1] * (double)sizes[k]));
        if (k && lo[k] <= lo[k - 1]) lo[k] = lo[k - 1] + 1;
    }
    planb_set_tuning(fib, &saved);
    if (rc != PLANB_OK) {
        fib->size_tunings.swap(keep);
        return rc;
    }
    return planb_set_size_tunings(fib, lo.data(), tu.data(), count);
}

}  // extern "C"
