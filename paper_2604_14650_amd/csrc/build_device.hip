// Device-side build: the elementary intervals and the tree image of
// planb_build computed on the GPU, so that a FIB can be rebuilt from its rule
// set next to the lookups (the paper rebuilds the whole structure on every
// update, Section 3.6, and swaps it in).
//
// The steps are those of the host build (range conversion, event sort, stack
// sweep and layout: Sections 3.1 and 3.2, Algorithm 2), restated for
// data-parallel hardware:
//  * events: one thread per rule masks its prefix and emits a START event at
//    the prefix and, unless the range ends at 2^128, an END event at the
//    exclusive end;
//  * sort: three stable radix sorts order the events by (address, END before
//    START, START by length), least significant field first (device_sort.hpp);
//  * sweep: the stack depth after each event is a prefix sum of +1 / -1.  The
//    top of the stack after event k is the START at the latest position
//    j <= k whose depth after it equals the depth after k: a later START at
//    that depth would be on top instead, and for an earlier one the depth
//    must have dropped below it (popping it) before returning.  The STARTs
//    are sorted by (depth, position) once, and the last event of each
//    address finds its top by binary search;
//  * intervals: one per distinct address, plus address 0 with NO_ROUTE when
//    no rule starts there, compacted by a prefix sum (and, with the merge
//    flag, a second compaction of equal neighbours);
//  * image: the slot array is filled with the sentinel, then the leaf keys
//    and next hops are scattered and the separators gathered level by level.
// The image, the intervals and the errors are those of the host build.
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "api_internal.hpp"
#include "device_sort.hpp"

namespace planb {
namespace {

constexpr uint16_t kTbDummy = 0xFFFF;  // no END event: sorts after every real event
constexpr int kThreads = 256;

struct BuildState {  // device-side results, read back once
    uint32_t bad_rule;      // smallest rule index with length > 128 or next hop 0xFFFF (~0u: none)
    uint32_t dup;           // some (prefix, length) repeated after masking
    uint32_t dummies;       // rules whose range ends at 2^128
    uint32_t any_lo;        // some interval start has a nonzero low word
    uint32_t any_mid;       // some interval start has nonzero bits 64..95
    uint32_t unbalanced;    // a negative stack depth (cannot happen for valid input)
    uint32_t zero_missing;  // no event at address 0
    uint64_t groups;        // distinct event addresses
    uint64_t m;             // intervals
};

__device__ inline void mask_range(uint64_t hi, uint64_t lo, int L, uint64_t* mhi, uint64_t* mlo, bool* has_end,
                                  uint64_t* ehi, uint64_t* elo)
{
    if (L == 0) {
        hi = lo = 0;
    } else if (L <= 64) {
        hi = L == 64 ? hi : (hi & ~(~0ull >> L));
        lo = 0;
    } else if (L < 128) {
        lo &= ~((1ull << (128 - L)) - 1);
    }
    *mhi = hi;
    *mlo = lo;
    // exclusive end hi:lo + 2^(128 - L); none when it reaches 2^128
    *has_end = false;
    if (L == 0) return;
    const int h = 128 - L;
    if (h >= 64) {
        const uint64_t r = hi + (1ull << (h - 64));
        if (r < hi) return;
        *ehi = r;
        *elo = lo;
    } else {
        const uint64_t r = lo + (1ull << h);
        const uint64_t carry = r < lo ? 1 : 0;
        const uint64_t rh = hi + carry;
        if (carry && rh == 0) return;
        *ehi = rh;
        *elo = r;
    }
    *has_end = true;
}

__global__ void events_kernel(const u64x2* __restrict__ prefixes, const uint8_t* __restrict__ lengths,
                              const uint16_t* __restrict__ nhs, uint32_t n, uint64_t* __restrict__ ev_hi,
                              uint64_t* __restrict__ ev_lo, uint16_t* __restrict__ ev_tb, uint32_t* __restrict__ ev_id,
                              BuildState* st)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int L0 = lengths[i];
    if (L0 > 128 || nhs[i] == kNoRoute) atomicMin(&st->bad_rule, i);
    const int L = L0 > 128 ? 128 : L0;
    const u64x2 p = prefixes[i];
    uint64_t hi, lo, ehi = 0, elo = 0;
    bool has_end;
    mask_range(p.x, p.y, L, &hi, &lo, &has_end, &ehi, &elo);
    ev_hi[2 * i] = hi;
    ev_lo[2 * i] = lo;
    ev_tb[2 * i] = (uint16_t)(256 + L);  // START: after ENDs, by length
    ev_id[2 * i] = i;
    if (has_end) {
        ev_hi[2 * i + 1] = ehi;
        ev_lo[2 * i + 1] = elo;
        ev_tb[2 * i + 1] = (uint16_t)L;  // END
    } else {
        ev_hi[2 * i + 1] = ~0ull;
        ev_lo[2 * i + 1] = ~0ull;
        ev_tb[2 * i + 1] = kTbDummy;
        atomicAdd(&st->dummies, 1u);
    }
    ev_id[2 * i + 1] = i;
}

template <typename T>
__global__ void gather_kernel(const T* __restrict__ src, const uint32_t* __restrict__ perm, uint32_t n, T* __restrict__ dst)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = src[perm[k]];
}

__global__ void iota_kernel(uint32_t* v, uint32_t n)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) v[k] = k;
}

// Per sorted event: depth step, "last event of its address", duplicate check,
// and the START key for the (depth, position) sort (filled in after the scan).
__global__ void mark_kernel(const uint64_t* __restrict__ hi, const uint64_t* __restrict__ lo,
                            const uint16_t* __restrict__ tb, uint32_t total, int32_t* __restrict__ delta,
                            uint32_t* __restrict__ last, BuildState* st)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= total) return;
    const uint32_t E = total - st->dummies;
    if (k >= E) {
        delta[k] = 0;
        last[k] = 0;
        return;
    }
    const bool start = tb[k] >= 256;
    delta[k] = start ? 1 : -1;
    last[k] = (k + 1 == E || hi[k + 1] != hi[k] || lo[k + 1] != lo[k]) ? 1u : 0u;
    if (k > 0 && start && tb[k - 1] == tb[k] && hi[k - 1] == hi[k] && lo[k - 1] == lo[k]) st->dup = 1;
    if (k == 0) st->zero_missing = (hi[0] != 0 || lo[0] != 0) ? 1u : 0u;
}

__global__ void start_keys_kernel(const uint16_t* __restrict__ tb, const int32_t* __restrict__ depth, uint32_t total,
                                  uint32_t* __restrict__ skey, BuildState* st)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= total) return;
    const uint32_t E = total - st->dummies;
    const bool start = k < E && tb[k] >= 256;
    if (k < E && depth[k] < 0) st->unbalanced = 1;
    skey[k] = start ? (uint32_t)depth[k] : ~0u;
}

// first index in [lo, hi) with a[i] >= v (a sorted ascending)
__device__ inline uint32_t lower_bound_u32(const uint32_t* a, uint32_t lo, uint32_t hi, uint32_t v)
{
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// One interval per address group (written at the group's last event).
__global__ void resolve_kernel(const uint64_t* __restrict__ hi, const uint64_t* __restrict__ lo,
                               const uint32_t* __restrict__ id, const int32_t* __restrict__ depth,
                               const uint32_t* __restrict__ last, const uint32_t* __restrict__ gpos,
                               const uint32_t* __restrict__ skey, const uint32_t* __restrict__ spos, uint32_t n_starts,
                               const uint16_t* __restrict__ nhs, uint32_t total, u64x2* __restrict__ starts,
                               uint16_t* __restrict__ nh_out, BuildState* st)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t E = total - st->dummies;
    const uint32_t z = st->zero_missing;
    if (k == 0) {
        if (z) {
            starts[0] = u64x2{0, 0};
            nh_out[0] = kNoRoute;
        }
        st->groups = E ? (uint64_t)gpos[E - 1] + last[E - 1] : 0;
    }
    if (k >= E || !last[k]) return;
    const int32_t d = depth[k];
    uint16_t nh = kNoRoute;
    if (d > 0) {
        const uint32_t a = lower_bound_u32(skey, 0, n_starts, (uint32_t)d);
        const uint32_t b = lower_bound_u32(skey, a, n_starts, (uint32_t)d + 1);
        // last position <= k among spos[a..b) (ascending: the sort is stable)
        uint32_t l = a, h = b;
        while (l < h) {
            const uint32_t mid = (l + h) >> 1;
            if (spos[mid] <= k) l = mid + 1; else h = mid;
        }
        if (l > a) nh = nhs[id[spos[l - 1]]];
        else st->unbalanced = 1;
    }
    const uint32_t p = gpos[k] + z;
    starts[p] = u64x2{hi[k], lo[k]};
    nh_out[p] = nh;
}

__global__ void keep_kernel(const uint16_t* __restrict__ nh, uint32_t m, uint32_t* __restrict__ keep)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) keep[i] = (i == 0 || nh[i] != nh[i - 1]) ? 1u : 0u;
}

__global__ void compact_kernel(const u64x2* __restrict__ starts, const uint16_t* __restrict__ nh, uint32_t m,
                               const uint32_t* __restrict__ keep, const uint32_t* __restrict__ kpos,
                               u64x2* __restrict__ starts2, uint16_t* __restrict__ nh2)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m && keep[i]) {
        starts2[kpos[i]] = starts[i];
        nh2[kpos[i]] = nh[i];
    }
}

__global__ void finish_kernel(const u64x2* __restrict__ starts, uint32_t m, BuildState* st)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) st->m = m;
    if (i < m && starts[i].y != 0) st->any_lo = 1;
    if (i < m && (starts[i].x & 0xFFFFFFFFull) != 0) st->any_mid = 1;
}

__global__ void count_kernel(const uint32_t* __restrict__ keep, const uint32_t* __restrict__ kpos, uint32_t m,
                             BuildState* st)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) st->m = m ? (uint64_t)kpos[m - 1] + keep[m - 1] : 0;
}

// A key in a slot of kb bytes: {hi, lo}, hi, or hi's top 32 bits.
__device__ inline void write_key(uint8_t* slot, u64x2 v, int kb)
{
    if (kb == 4) {
        *reinterpret_cast<uint32_t*>(slot) = (uint32_t)(v.x >> 32);
    } else {
        reinterpret_cast<uint64_t*>(slot)[0] = v.x;
        if (kb == 16) reinterpret_cast<uint64_t*>(slot)[1] = v.y;
    }
}

// Leaf keys and next hops.
__global__ void leaves_kernel(const u64x2* __restrict__ starts, const uint16_t* __restrict__ nh, uint32_t m, int kb,
                              uint32_t lc, uint32_t ls, uint64_t leaf_base, uint8_t* __restrict__ image)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const uint32_t q = i / lc, s = i % lc;
    uint8_t* leaf = image + (leaf_base + (uint64_t)q * ls) * kb;
    write_key(leaf + (uint64_t)leaf_key_slot(s, kb) * kb, starts[i], kb);
    *reinterpret_cast<uint16_t*>(leaf + leaf_hop_byte(s, kb, (int)lc)) = nh[i];
}

// Separators of one internal level: slot j-1 of node q = the first key of the
// leaf that starts child j's subtree (q*b + j) * span, if that leaf exists.
__global__ void separators_kernel(const u64x2* __restrict__ starts, uint64_t nodes, uint64_t node_off, uint32_t b,
                                  uint64_t span, uint64_t leaves, uint32_t lc, int kb, uint8_t* __restrict__ image)
{
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nodes * (b - 1)) return;
    const uint64_t q = t / (b - 1), j = t % (b - 1) + 1;
    const uint64_t leaf = (q * b + j) * span;
    if (leaf >= leaves) return;
    write_key(image + ((node_off + q) * b + j - 1) * kb, starts[leaf * lc], kb);
}

unsigned blocks_for(uint64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

// Device buffers of one build, freed on every exit.
struct Scratch {
    std::vector<void*> ptrs;
    ~Scratch()
    {
        for (void* p : ptrs) (void)hipFree(p);
    }
    template <typename T>
    hipError_t get(T** p, size_t count)
    {
        *p = nullptr;
        hipError_t e = hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(count, 1) * sizeof(T));
        if (e == hipSuccess) ptrs.push_back(*p);
        return e;
    }
};

#define PB_TRY(call)                          \
    do {                                      \
        hipError_t e_ = (call);               \
        if (e_ != hipSuccess) return e_;      \
    } while (0)

template <typename K, typename V>
hipError_t sort_pairs(Scratch& S, const K* kin, K* kout, const V* vin, V* vout, uint32_t n, unsigned bits,
                      hipStream_t st)
{
    auto alloc = [&](void** p, size_t bytes) { return S.get(reinterpret_cast<uint8_t**>(p), bytes); };
    return dsort::sort_pairs(alloc, kin, kout, vin, vout, n, bits, st);
}

template <typename T>
hipError_t scan(Scratch& S, const T* in, T* out, uint32_t n, bool inclusive, hipStream_t st)
{
    auto alloc = [&](void** p, size_t bytes) { return S.get(reinterpret_cast<uint8_t**>(p), bytes); };
    return dsort::scan<T>(alloc, in, out, n, inclusive, st);
}

// Intervals of n rules (device arrays), before any merge, into out_starts /
// out_nh (capacity 2n + 1 each).
hipError_t device_intervals(Scratch& S, const u64x2* prefixes, const uint8_t* lengths, const uint16_t* nhs,
                            uint32_t n, u64x2* out_starts, uint16_t* out_nh, BuildState* d_st, hipStream_t st)
{
    const uint32_t total = 2 * n;
    uint64_t *ev_hi, *ev_lo, *hi_a, *hi_b;
    uint16_t *ev_tb, *tb_s;
    uint32_t *ev_id, *perm_a, *perm_b, *id_s, *last, *gpos, *skey, *skey_s, *pos, *spos;
    int32_t *delta, *depth;
    PB_TRY(S.get(&ev_hi, total));
    PB_TRY(S.get(&ev_lo, total));
    PB_TRY(S.get(&hi_a, total));
    PB_TRY(S.get(&hi_b, total));
    PB_TRY(S.get(&ev_tb, total));
    PB_TRY(S.get(&tb_s, total));
    PB_TRY(S.get(&ev_id, total));
    PB_TRY(S.get(&perm_a, total));
    PB_TRY(S.get(&perm_b, total));
    PB_TRY(S.get(&id_s, total));
    PB_TRY(S.get(&last, total));
    PB_TRY(S.get(&gpos, total));
    PB_TRY(S.get(&skey, total));
    PB_TRY(S.get(&skey_s, total));
    PB_TRY(S.get(&pos, total));
    PB_TRY(S.get(&spos, total));
    PB_TRY(S.get(&delta, total));
    PB_TRY(S.get(&depth, total));
    const unsigned g = blocks_for(total);
    hipLaunchKernelGGL(events_kernel, dim3(blocks_for(n)), dim3(kThreads), 0, st, prefixes, lengths, nhs, n, ev_hi,
                       ev_lo, ev_tb, ev_id, d_st);
    PB_TRY(hipGetLastError());
    // stable LSD passes: (type, length), then the low word, then the high word
    hipLaunchKernelGGL(iota_kernel, dim3(g), dim3(kThreads), 0, st, perm_b, total);
    PB_TRY(sort_pairs(S, ev_tb, tb_s, perm_b, perm_a, total, 16, st));
    hipLaunchKernelGGL(gather_kernel<uint64_t>, dim3(g), dim3(kThreads), 0, st, ev_lo, perm_a, total, hi_a);
    PB_TRY(sort_pairs(S, hi_a, hi_b, perm_a, perm_b, total, 64, st));  // hi_b: sorted low words (scratch)
    hipLaunchKernelGGL(gather_kernel<uint64_t>, dim3(g), dim3(kThreads), 0, st, ev_hi, perm_b, total, hi_a);
    PB_TRY(sort_pairs(S, hi_a, hi_b, perm_b, perm_a, total, 64, st));  // hi_b: sorted high words
    // final order perm_a: the other fields follow it
    uint64_t* lo_s = hi_a;
    hipLaunchKernelGGL(gather_kernel<uint64_t>, dim3(g), dim3(kThreads), 0, st, ev_lo, perm_a, total, lo_s);
    hipLaunchKernelGGL(gather_kernel<uint16_t>, dim3(g), dim3(kThreads), 0, st, ev_tb, perm_a, total, tb_s);
    hipLaunchKernelGGL(gather_kernel<uint32_t>, dim3(g), dim3(kThreads), 0, st, ev_id, perm_a, total, id_s);
    const uint64_t* hi_s = hi_b;
    hipLaunchKernelGGL(mark_kernel, dim3(g), dim3(kThreads), 0, st, hi_s, lo_s, tb_s, total, delta, last, d_st);
    PB_TRY(hipGetLastError());
    PB_TRY(scan(S, delta, depth, total, true, st));
    PB_TRY(scan(S, last, gpos, total, false, st));
    hipLaunchKernelGGL(start_keys_kernel, dim3(g), dim3(kThreads), 0, st, tb_s, depth, total, skey, d_st);
    hipLaunchKernelGGL(iota_kernel, dim3(g), dim3(kThreads), 0, st, pos, total);
    PB_TRY(sort_pairs(S, skey, skey_s, pos, spos, total, 32, st));
    hipLaunchKernelGGL(resolve_kernel, dim3(g), dim3(kThreads), 0, st, hi_s, lo_s, id_s, depth, last, gpos, skey_s,
                       spos, n, nhs, total, out_starts, out_nh, d_st);
    PB_TRY(hipGetLastError());
    return hipSuccess;
}

}  // namespace
}  // namespace planb

using namespace planb;

extern "C" planb_fib_t* planb_build_device(const planb_addr_t* prefixes, const uint8_t* lengths,
                                           const uint16_t* next_hops, size_t n, const planb_params_t* params,
                                           void* stream)
{
    clear_error();
    planb_params_t p{};
    if (params) p = *params;
    if (p.fanout == 0) p.fanout = 16;
    if (p.fanout != 8 && p.fanout != 16 && p.fanout != 32) {
        fail(PLANB_EINVAL, "fanout must be 8, 16 or 32");
        return nullptr;
    }
    if (p.key_bits != 0 && p.key_bits != 32 && p.key_bits != 64 && p.key_bits != 128) {
        fail(PLANB_EINVAL, "key_bits must be 0, 32, 64 or 128");
        return nullptr;
    }
    if (n > 0 && (!prefixes || !lengths || !next_hops)) {
        fail(PLANB_EINVAL, "NULL input array with n > 0");
        return nullptr;
    }
    if (reinterpret_cast<uintptr_t>(prefixes) % 16 || reinterpret_cast<uintptr_t>(next_hops) % 2) {
        fail(PLANB_EINVAL, "prefixes must be 16-byte and next_hops 2-byte aligned");
        return nullptr;
    }
    if (n >= (1ull << 30)) {
        fail(PLANB_ERANGE, "too many rules for the device build (at most 2^30 - 1)");
        return nullptr;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    planb_fib_t* f = new (std::nothrow) planb_fib_t();
    if (!f) {
        fail(PLANB_ENOMEM, "out of host memory");
        return nullptr;
    }
    auto bail = [&](int code, const std::string& msg) -> planb_fib_t* {
        fail(code, msg);
        planb_free(f);
        return nullptr;
    };
    if (hipGetDevice(&f->device) != hipSuccess) return bail(PLANB_EDEVICE, "hipGetDevice failed");
    const uint32_t nn = (uint32_t)n;
    Scratch S;
    BuildState* d_st = nullptr;
    u64x2* d_starts = nullptr;
    uint16_t* d_nh = nullptr;
    hipError_t e;
    BuildState h{};
    if ((e = S.get(&d_st, 1)) != hipSuccess || (e = S.get(&d_starts, 2 * (size_t)nn + 1)) != hipSuccess ||
        (e = S.get(&d_nh, 2 * (size_t)nn + 1)) != hipSuccess)
        return bail(PLANB_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    h.bad_rule = ~0u;
    if ((e = hipMemcpyAsync(d_st, &h, sizeof(h), hipMemcpyHostToDevice, st)) != hipSuccess)
        return bail(PLANB_EDEVICE, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
    const bool merge = (p.flags & PLANB_FLAG_MERGE_EQUAL_NH) != 0;
    u64x2* un_starts = d_starts;  // intervals before the optional merge
    uint16_t* un_nh = d_nh;
    if (merge && nn && ((e = S.get(&un_starts, 2 * (size_t)nn + 1)) != hipSuccess ||
                        (e = S.get(&un_nh, 2 * (size_t)nn + 1)) != hipSuccess))
        return bail(PLANB_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    static const u64x2 kZero{0, 0};
    static const uint16_t kNone = kNoRoute;
    if (nn == 0) {  // one interval, the whole space, NO_ROUTE
        if ((e = hipMemcpyAsync(d_starts, &kZero, sizeof(kZero), hipMemcpyHostToDevice, st)) != hipSuccess ||
            (e = hipMemcpyAsync(d_nh, &kNone, 2, hipMemcpyHostToDevice, st)) != hipSuccess)
            return bail(PLANB_EDEVICE, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
    } else {
        if ((e = device_intervals(S, reinterpret_cast<const u64x2*>(prefixes), lengths, next_hops, nn, un_starts,
                                  un_nh, d_st, st)) != hipSuccess)
            return bail(e == hipErrorOutOfMemory ? PLANB_ENOMEM : PLANB_EDEVICE,
                        std::string("device build: ") + hipGetErrorString(e));
    }
    // interval count (m0 before the optional merge) and errors
    if ((e = hipMemcpyAsync(&h, d_st, sizeof(h), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return bail(PLANB_EDEVICE, std::string("device build: ") + hipGetErrorString(e));
    if (h.bad_rule != ~0u) {
        uint8_t L = 0;
        uint16_t v = 0;
        (void)hipMemcpy(&L, lengths + h.bad_rule, 1, hipMemcpyDeviceToHost);
        (void)hipMemcpy(&v, next_hops + h.bad_rule, 2, hipMemcpyDeviceToHost);
        return bail(PLANB_EINVAL, L > 128 ? "prefix length " + std::to_string(L) + " > 128 at rule " +
                                                std::to_string(h.bad_rule)
                                          : "next hop 0xFFFF (reserved for NO_ROUTE) at rule " +
                                                std::to_string(h.bad_rule));
    }
    if (h.dup) return bail(PLANB_EDUP, "duplicate rule after masking host bits");
    if (h.unbalanced) return bail(PLANB_EDEVICE, "internal error: unbalanced interval sweep");
    uint64_t m = nn ? h.groups + h.zero_missing : 1;
    if (merge && nn) {  // keep the first of every run of equal next hops
        uint32_t *keep, *kpos;
        if ((e = S.get(&keep, m)) != hipSuccess || (e = S.get(&kpos, m)) != hipSuccess)
            return bail(PLANB_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        hipLaunchKernelGGL(keep_kernel, dim3(blocks_for(m)), dim3(kThreads), 0, st, un_nh, (uint32_t)m, keep);
        if ((e = scan(S, keep, kpos, (uint32_t)m, false, st)) != hipSuccess)
            return bail(PLANB_EDEVICE, std::string("device build: ") + hipGetErrorString(e));
        hipLaunchKernelGGL(compact_kernel, dim3(blocks_for(m)), dim3(kThreads), 0, st, un_starts, un_nh, (uint32_t)m,
                           keep, kpos, d_starts, d_nh);
        hipLaunchKernelGGL(count_kernel, dim3(1), dim3(1), 0, st, keep, kpos, (uint32_t)m, d_st);
        if ((e = hipMemcpyAsync(&h.m, &d_st->m, 8, hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess)
            return bail(PLANB_EDEVICE, std::string("device build: ") + hipGetErrorString(e));
        m = h.m;
    }
    hipLaunchKernelGGL(finish_kernel, dim3(blocks_for(m)), dim3(kThreads), 0, st, d_starts, (uint32_t)m, d_st);
    uint32_t flags[2] = {0, 0};  // any_lo, any_mid
    if ((e = hipMemcpyAsync(flags, &d_st->any_lo, 8, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return bail(PLANB_EDEVICE, std::string("device build: ") + hipGetErrorString(e));
    int kb = 16;
    if (choose_key_bytes(flags[0] == 0, flags[0] == 0 && flags[1] == 0, p.key_bits, &kb) != PLANB_OK) {
        planb_free(f);
        return nullptr;
    }
    f->key_bytes_per_slot = (uint32_t)kb;
    std::string err;
    int rc = plan_fib_layout(m, p.fanout, kb, &f->lay, &err);
    if (rc != 0) return bail(rc == -5 ? PLANB_ERANGE : PLANB_EINVAL, err);
    const Layout& lay = f->lay;
    const size_t kbytes = lay.total_slots() * kb, vbytes = ((m + 63) / 64) * 64 * sizeof(uint16_t);
    if ((e = fib_alloc(f->device, &f->d_keys, kbytes)) != hipSuccess ||
        (e = fib_alloc(f->device, reinterpret_cast<void**>(&f->d_vals), vbytes)) != hipSuccess)
        return bail(PLANB_ENOMEM, std::string("device allocation: ") + hipGetErrorString(e));
    f->key_bytes = kbytes;
    f->value_bytes = vbytes;
    uint8_t* img = static_cast<uint8_t*>(f->d_keys);
    if ((e = hipMemsetAsync(img, 0xFF, kbytes, st)) != hipSuccess ||
        (e = hipMemsetAsync(f->d_vals, 0xFF, vbytes, st)) != hipSuccess ||
        (e = hipMemcpyAsync(f->d_vals, d_nh, m * 2, hipMemcpyDeviceToDevice, st)) != hipSuccess)
        return bail(PLANB_EDEVICE, std::string("device build: ") + hipGetErrorString(e));
    hipLaunchKernelGGL(leaves_kernel, dim3(blocks_for(m)), dim3(kThreads), 0, st, d_starts, d_nh, (uint32_t)m, kb,
                       lay.leaf_cap, lay.leaf_slots, (uint64_t)lay.leaf_base(), img);
    uint64_t span = 1;  // leaves under one node of level l + 1
    for (int l = (int)lay.depth - 2; l >= 0; --l) {
        const uint64_t work = lay.nodes[l] * (lay.b - 1);
        hipLaunchKernelGGL(separators_kernel, dim3(blocks_for(work)), dim3(kThreads), 0, st, d_starts, lay.nodes[l],
                           lay.offset[l], lay.b, span, lay.leaves, lay.leaf_cap, kb, img);
        span *= lay.b;
    }
    if ((e = hipGetLastError()) != hipSuccess)
        return bail(PLANB_EDEVICE, std::string("device build: ") + hipGetErrorString(e));
    // host copy of the intervals (export, learned training, the server's accounting)
    try {
        f->iv.starts.resize(m);
        f->iv.nh.resize(m);
    } catch (const std::bad_alloc&) {
        return bail(PLANB_ENOMEM, "out of host memory");
    }
    if ((e = hipMemcpyAsync(f->iv.starts.data(), d_starts, m * 16, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipMemcpyAsync(f->iv.nh.data(), d_nh, m * 2, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return bail(PLANB_EDEVICE, std::string("device build: ") + hipGetErrorString(e));
    if (finish_fib(f, p) != PLANB_OK) {
        planb_free(f);
        return nullptr;
    }
    return f;
}
