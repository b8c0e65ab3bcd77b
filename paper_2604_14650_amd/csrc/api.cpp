// C ABI of the library (declared in include/planb.h).
#include "api_internal.hpp"

#include <algorithm>
#include <cstring>
#include <new>

using namespace planb;

namespace planb {

thread_local std::string g_err;
thread_local int g_status = 0;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    g_status = code;
    return code;
}

int fail_hip(hipError_t e, const char* what)
{
    return fail(PLANB_EDEVICE, std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")");
}

int check_current_device(const planb_fib_t* fib)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    if (dev != fib->device)
        return fail(PLANB_EINVAL, "the FIB lives on device " + std::to_string(fib->device) +
                                      " but device " + std::to_string(dev) + " is current");
    return PLANB_OK;
}

int deepest_lds_levels(const Layout& lay, size_t key_bytes, size_t budget)
{
    int L = 0;
    while (L < (int)lay.depth && lay.prefix_slots(L + 1) * key_bytes <= budget) ++L;
    return L;
}

TreeDesc make_desc(const planb_fib_t* f, int32_t lds_levels)
{
    TreeDesc t{};
    t.keys = f->d_keys;
    t.key_bytes = f->key_bytes_per_slot;
    t.vals = f->d_vals;
    t.m_minus_1 = f->iv.starts.size() - 1;
    t.depth = f->lay.depth;
    t.lds_levels = (uint32_t)lds_levels;
    t.lds_slots = (uint32_t)f->lay.prefix_slots(lds_levels);
    t.fanout = f->lay.b;
    t.leaf_base = (uint32_t)f->lay.leaf_base();
    t.last_hop = f->iv.nh.empty() ? 0xFFFFu : f->iv.nh.back();
    for (int l = 0; l < kDevMaxLevels; ++l) {
        t.off[l] = l < (int)f->lay.depth ? (uint32_t)f->lay.offset[l] : 0;
        t.last[l] = l < (int)f->lay.depth ? (uint32_t)(f->lay.nodes[l] - 1) : 0;
    }
    return t;
}

void refresh_desc(planb_fib_t* f)
{
    f->desc = make_desc(f, f->lds_levels);
    for (auto& s : f->size_tunings) s.desc = make_desc(f, s.lds_levels);
}

void shape_for(const planb_fib_t* f, uint64_t n, const LookupTuning** tu, const TreeDesc** desc)
{
    *tu = &f->tune;
    *desc = &f->desc;
    for (const auto& s : f->size_tunings) {
        if (s.min_lookups > n) break;
        *tu = &s.tune;
        *desc = &s.desc;
    }
}

int validate_tuning(const planb_fib_t* f, const planb_tuning_t& tu, LookupTuning* out, int32_t* lds_out)
{
    const uint32_t b = f->lay.b, kpl = tu.keys_per_lane, R = tu.lookups_per_group, bs = tu.block_threads;
    const bool bin = tu.lds_search != 0, tops = tu.lds_search == 2;
    if (kpl == 0 || (kpl & (kpl - 1)) || b % kpl || b / kpl > 32 || (bs != 512 && bs != 1024) ||
        tu.lds_search > 2 || (bin && kpl != b && b / kpl != 2 && b / kpl != 4) ||
        !lookup_variant_exists((int)b, (int)kpl, (int)R, (int)bs, bin))
        return fail(PLANB_EINVAL, "unsupported tuning: keys_per_lane " + std::to_string(kpl) +
                                      ", lookups_per_group " + std::to_string(R) + ", block_threads " +
                                      std::to_string(bs) + " for fanout " + std::to_string(b));
    if (tops) {
        const uint32_t kb = f->key_bytes_per_slot;
        if ((kb != 8 && kb != 16) || kpl == b || !lookup_tops_variant_exists((int)b, (int)kpl, (int)R, (int)kb, (int)bs))
            return fail(PLANB_EINVAL, "lds_search 2 needs 64- or 128-bit key slots and fanout / keys_per_lane of 2 or 4");
        // exact levels above the bottom internal one, then that level's key tops (b - 1 per node)
        const uint32_t D = f->lay.depth;
        const size_t tb = D < 2 ? 0
                                : f->lay.prefix_slots(D - 2) * (size_t)kb +
                                      (size_t)f->lay.nodes[D - 2] * (b - 1) * 4;
        if (tb > (size_t)max_lds_bytes())
            return fail(PLANB_ERANGE, "the internal levels with the bottom one as key tops need " + std::to_string(tb) +
                                          " bytes of LDS, more than a workgroup may allocate");
    }
    int32_t lds_levels = tu.lds_levels;
    if (lds_levels < 0) lds_levels = deepest_lds_levels(f->lay, f->key_bytes_per_slot, 64 * 1024);
    if (lds_levels > (int32_t)f->lay.depth) return fail(PLANB_EINVAL, "lds_levels exceeds the tree depth");
    const size_t bytes = f->lay.prefix_slots(lds_levels) * (size_t)f->key_bytes_per_slot;
    if (bytes > (size_t)max_lds_bytes())
        return fail(PLANB_ERANGE, "the top " + std::to_string(lds_levels) + " levels need " + std::to_string(bytes) +
                                      " bytes of LDS, more than a workgroup may allocate");
    out->kpl = (int)kpl;
    out->R = (int)R;
    out->block = (int)bs;
    out->bin = bin;
    out->tops = tops;
    *lds_out = lds_levels;
    return PLANB_OK;
}

void layout_to_info(const Layout& lay, planb_info_t* info)
{
    std::memset(info, 0, sizeof(*info));
    info->intervals = lay.m;
    info->fanout = lay.b;
    info->slots = lay.slots;
    info->depth = lay.depth;
    for (uint32_t l = 0; l < lay.depth; ++l) info->level_nodes[l] = lay.nodes[l];
    for (uint32_t l = 0; l <= lay.depth; ++l) info->level_offset[l] = lay.offset[l];
    info->key_bits = 128;
    info->key_bytes = lay.total_slots() * 16ull;
    info->leaf_keys = lay.leaf_cap;
    info->leaf_slots = lay.leaf_slots;
    info->leaf_base = lay.leaf_base();
}

void clear_error()
{
    g_err.clear();
    g_status = 0;
}

uint32_t default_kpl(uint32_t b) { return b == 8 ? 2 : b == 16 ? 4 : 8; }

int plan_fib_layout(uint64_t m, uint32_t fanout, int key_bytes, Layout* lay, std::string* err)
{
    const int rc = plan_layout(m, fanout, fanout, (uint32_t)leaf_cap_for((int)fanout, key_bytes),
                               (uint32_t)leaf_slots_for((int)fanout, key_bytes), true, lay, err);
    // the kernels address the slot array with 32-bit byte offsets
    if (rc == 0 && lay->total_slots() * (uint64_t)key_bytes > UINT32_MAX) {
        *err = "tree image of " + std::to_string(lay->total_slots() * (uint64_t)key_bytes) +
               " bytes: the slot array must stay below 4 GiB";
        return -5;
    }
    return rc;
}

// The device slot array of a FIB: the keys of fill_keys in key_bytes-wide
// slots (8: the hi word of every key, 4: its top 32 bits), and each leaf's next hops written
// where the leaf format puts them (kNoRoute past the last interval).
void build_image(const Intervals& iv, const Layout& lay, int key_bytes, std::vector<uint8_t>* image)
{
    std::vector<U128> keys;
    fill_keys(iv, lay, key_bytes, &keys);
    image->assign(keys.size() * key_bytes, 0);
    if (key_bytes == 4) {
        uint32_t* d = reinterpret_cast<uint32_t*>(image->data());
        for (size_t i = 0; i < keys.size(); ++i) d[i] = (uint32_t)(keys[i].hi >> 32);
    } else if (key_bytes == 8) {
        uint64_t* d = reinterpret_cast<uint64_t*>(image->data());
        for (size_t i = 0; i < keys.size(); ++i) d[i] = keys[i].hi;
    } else {
        std::memcpy(image->data(), keys.data(), image->size());
    }
    const uint64_t m = iv.starts.size(), LC = lay.leaf_cap, LS = lay.leaf_slots, base = lay.leaf_base();
    for (uint64_t q = 0; q < lay.leaves; ++q) {
        uint8_t* leaf = image->data() + (base + q * LS) * key_bytes;
        for (uint64_t s = 0; s < LC; ++s) {
            const uint64_t i = q * LC + s;
            const uint16_t v = i < m ? iv.nh[i] : kNoRoute;
            std::memcpy(leaf + leaf_hop_byte((uint32_t)s, key_bytes, (int)LC), &v, 2);
        }
    }
}

int finish_fib(planb_fib_t* f, const planb_params_t& p)
{
    // The initial launch shape, the fastest that applies of the measured
    // ones: the key tops (1024 threads), else the hybrid binary search, else
    // every lane comparing its keys (512 threads).
    planb_tuning_t tu{};
    tu.keys_per_lane = p.keys_per_lane ? p.keys_per_lane : default_kpl(p.fanout);
    tu.lds_levels = p.lds_levels > 0 ? p.lds_levels : -1;
    tu.lookups_per_group = 2;
    int32_t lds_ok = 0;
    int rc = PLANB_EINVAL;
    for (uint32_t mode : {2u, 1u, 0u}) {
        tu.lds_search = mode;
        tu.block_threads = mode == 2 ? 1024 : 512;
        if ((rc = validate_tuning(f, tu, &f->tune, &lds_ok)) == PLANB_OK) break;
    }
    if (rc != PLANB_OK) return rc;
    clear_error();  // a shape that did not apply is no error of the build
    f->lds_levels = lds_ok;
    refresh_desc(f);
    return PLANB_OK;
}

// Key width for a set of interval starts: the width asked for when it is
// exact, else (nothing asked) the narrowest exact one: 4 bytes when every
// start's low 96 bits are zero, 8 when every low word is zero, else 16.
int choose_key_bytes(bool lo_zero, bool low96_zero, uint32_t key_bits, int* key_bytes)
{
    if (key_bits != 0 && key_bits != 32 && key_bits != 64 && key_bits != 128)
        return fail(PLANB_EINVAL, "key_bits must be 0, 32, 64 or 128");
    if (key_bits == 64 && !lo_zero)
        return fail(PLANB_EINVAL, "64-bit keys are exact only when every interval start has a zero low word");
    if (key_bits == 32 && !low96_zero)
        return fail(PLANB_EINVAL, "32-bit keys are exact only when every interval start has zero low 96 bits");
    *key_bytes = key_bits == 32 ? 4 : key_bits == 64 ? 8 : key_bits == 128 ? 16 : low96_zero ? 4 : lo_zero ? 8 : 16;
    return PLANB_OK;
}

int choose_key_bytes(const Intervals& iv, uint32_t key_bits, int* key_bytes)
{
    bool lo_zero = true, low96_zero = true;
    for (const U128& k : iv.starts) {
        lo_zero &= (k.lo == 0);
        low96_zero &= (k.lo == 0 && (k.hi & 0xFFFFFFFFull) == 0);
    }
    return choose_key_bytes(lo_zero, low96_zero, key_bits, key_bytes);
}

}  // namespace planb

extern "C" {

const char* planb_last_error(void) { return g_err.c_str(); }

int planb_last_status(void) { return g_status; }

planb_fib_t* planb_build_ex(const planb_addr_t* prefixes, const uint8_t* lengths, const uint16_t* next_hops,
                            size_t n, const planb_params_t* params)
{
    clear_error();
    planb_params_t p{};
    if (params) p = *params;
    if (p.fanout == 0) p.fanout = 16;
    if (p.fanout != 8 && p.fanout != 16 && p.fanout != 32) {
        fail(PLANB_EINVAL, "fanout must be 8, 16 or 32");
        return nullptr;
    }
    if (n > 0 && (!prefixes || !lengths || !next_hops)) {
        fail(PLANB_EINVAL, "NULL input array with n > 0");
        return nullptr;
    }
    planb_fib_t* f = new (std::nothrow) planb_fib_t();
    if (!f) {
        fail(PLANB_ENOMEM, "out of host memory");
        return nullptr;
    }
    std::string err;
    int rc;
    try {
        rc = make_intervals(reinterpret_cast<const U128*>(prefixes), lengths, next_hops, n,
                            (p.flags & PLANB_FLAG_MERGE_EQUAL_NH) != 0, &f->iv, &err);
    } catch (const std::bad_alloc&) {
        rc = PLANB_ENOMEM;
        err = "out of host memory";
    }
    if (rc != 0) {
        fail(rc, err);
        delete f;
        return nullptr;
    }
    const uint64_t m = f->iv.starts.size();
    if (m >= (1ull << 31)) {
        fail(PLANB_ERANGE, "too many intervals (at most 2^31 - 1)");
        delete f;
        return nullptr;
    }
    int kb = 16;
    if ((rc = choose_key_bytes(f->iv, p.key_bits, &kb)) != PLANB_OK) {
        delete f;
        return nullptr;
    }
    f->key_bytes_per_slot = (uint32_t)kb;
    if ((rc = plan_fib_layout(m, p.fanout, kb, &f->lay, &err)) != 0) {
        fail(rc == -5 ? PLANB_ERANGE : PLANB_EINVAL, err);
        delete f;
        return nullptr;
    }
    std::vector<uint8_t> image;  // the device slot array, leaves carrying their next hops
    try {
        build_image(f->iv, f->lay, kb, &image);
    } catch (const std::bad_alloc&) {
        fail(PLANB_ENOMEM, "out of host memory");
        delete f;
        return nullptr;
    }
    hipError_t e = hipGetDevice(&f->device);
    if (e != hipSuccess) {
        fail_hip(e, "hipGetDevice");
        delete f;
        return nullptr;
    }
    const size_t kbytes = image.size();
    const size_t vbytes = ((m + 63) / 64) * 64 * sizeof(uint16_t);
    if ((e = fib_alloc(f->device, &f->d_keys, kbytes)) != hipSuccess ||
        (e = fib_alloc(f->device, reinterpret_cast<void**>(&f->d_vals), vbytes)) != hipSuccess) {
        fail(PLANB_ENOMEM, std::string("device allocation: ") + hipGetErrorString(e));
        planb_free(f);
        return nullptr;
    }
    f->key_bytes = kbytes;
    f->value_bytes = vbytes;
    if ((e = hipMemcpy(f->d_keys, image.data(), kbytes, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemset(f->d_vals, 0xFF, vbytes)) != hipSuccess ||
        (e = hipMemcpy(f->d_vals, f->iv.nh.data(), m * sizeof(uint16_t), hipMemcpyHostToDevice)) != hipSuccess) {
        fail_hip(e, "uploading the tree");
        planb_free(f);
        return nullptr;
    }
    if (finish_fib(f, p) != PLANB_OK) {
        planb_free(f);
        return nullptr;
    }
    return f;
}

planb_fib_t* planb_build(const planb_addr_t* prefixes, const uint8_t* lengths, const uint16_t* next_hops,
                         size_t n)
{
    return planb_build_ex(prefixes, lengths, next_hops, n, nullptr);
}

void planb_free(planb_fib_t* fib)
{
    if (!fib) return;
    release_learned(fib);
    free_after(fib->uses, fib->device, {fib->d_keys, fib->d_vals});
    delete fib;
}

static int check_lookup_args(const planb_fib_t* fib, const void* addrs, size_t n, const void* out,
                             size_t out_align)
{
    if (!fib) return fail(PLANB_EINVAL, "NULL fib");
    if (n == 0) return PLANB_OK;
    if (n >= (1ull << 40)) return fail(PLANB_ERANGE, "batch too large (n must be < 2^40)");
    if (!addrs || !out) return fail(PLANB_EINVAL, "NULL device pointer");
    if (reinterpret_cast<uintptr_t>(addrs) % 16) return fail(PLANB_EINVAL, "addrs must be 16-byte aligned");
    if (reinterpret_cast<uintptr_t>(out) % out_align) return fail(PLANB_EINVAL, "out is misaligned");
    return check_current_device(fib);
}

int planb_lookup(const planb_fib_t* fib, const planb_addr_t* addrs, size_t n, uint16_t* out, void* stream)
{
    int rc = check_lookup_args(fib, addrs, n, out, 2);
    if (rc != PLANB_OK || n == 0) return rc;
    const LookupTuning* tu;
    const TreeDesc* desc;
    shape_for(fib, n, &tu, &desc);
    hipError_t e = launch_lookup(*desc, *tu, addrs, n, out, false, static_cast<hipStream_t>(stream));
    if (e == hipSuccess) note_use(fib->uses, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? PLANB_OK : fail_hip(e, "lookup launch");
}

int planb_lookup_v4(const planb_fib_t* fib, const uint32_t* addrs, size_t n, uint16_t* out, void* stream)
{
    if (!fib) return fail(PLANB_EINVAL, "NULL fib");
    if (fib->key_bytes_per_slot != 4)
        return fail(PLANB_EINVAL, "the FIB's keys are not 32-bit: build it from rules of at most /32 placed in the top "
                                  "32 bits (key_bits 0 or 32)");
    if (n == 0) return PLANB_OK;
    if (n >= (1ull << 40)) return fail(PLANB_ERANGE, "batch too large (n must be < 2^40)");
    if (!addrs || !out) return fail(PLANB_EINVAL, "NULL device pointer");
    if (reinterpret_cast<uintptr_t>(addrs) % 4 || reinterpret_cast<uintptr_t>(out) % 2)
        return fail(PLANB_EINVAL, "misaligned pointer");
    int rc = check_current_device(fib);
    if (rc != PLANB_OK) return rc;
    hipError_t e = launch_lookup_v4(fib->desc, fib->tune, addrs, n, out, false, static_cast<hipStream_t>(stream));
    if (e == hipSuccess) note_use(fib->uses, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? PLANB_OK : fail_hip(e, "IPv4 lookup launch");
}

int planb_lookup_index(const planb_fib_t* fib, const planb_addr_t* addrs, size_t n, uint32_t* out, void* stream)
{
    int rc = check_lookup_args(fib, addrs, n, out, 4);
    if (rc != PLANB_OK || n == 0) return rc;
    const LookupTuning* tu;
    const TreeDesc* desc;
    shape_for(fib, n, &tu, &desc);
    hipError_t e = launch_lookup(*desc, *tu, addrs, n, out, true, static_cast<hipStream_t>(stream));
    if (e == hipSuccess) note_use(fib->uses, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? PLANB_OK : fail_hip(e, "lookup launch");
}

int planb_lookup_bsearch(const planb_fib_t* fib, const planb_addr_t* addrs, size_t n, uint16_t* out, void* stream)
{
    int rc = check_lookup_args(fib, addrs, n, out, 2);
    if (rc != PLANB_OK || n == 0) return rc;
    hipError_t e = launch_bsearch(fib->desc, addrs, n, out, static_cast<hipStream_t>(stream));
    if (e == hipSuccess) note_use(fib->uses, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? PLANB_OK : fail_hip(e, "binary-search launch");
}

size_t planb_num_intervals(const planb_fib_t* fib) { return fib ? fib->iv.starts.size() : 0; }

long long planb_export_intervals(const planb_fib_t* fib, planb_addr_t* starts, uint16_t* next_hops, size_t cap)
{
    if (!fib) return fail(PLANB_EINVAL, "NULL fib");
    const size_t m = std::min(cap, fib->iv.starts.size());
    if (starts) std::memcpy(starts, fib->iv.starts.data(), m * sizeof(planb_addr_t));
    if (next_hops) std::memcpy(next_hops, fib->iv.nh.data(), m * sizeof(uint16_t));
    return (long long)m;
}


long long planb_export_image(const planb_fib_t* fib, void* image, size_t cap_bytes)
{
    if (!fib) return fail(PLANB_EINVAL, "NULL fib");
    if (!image || cap_bytes < fib->key_bytes) return (long long)fib->key_bytes;
    int rc = check_current_device(fib);
    if (rc != PLANB_OK) return rc;
    hipError_t e = hipMemcpy(image, fib->d_keys, fib->key_bytes, hipMemcpyDeviceToHost);
    return e == hipSuccess ? (long long)fib->key_bytes : fail_hip(e, "copying the tree image");
}

long long planb_build_intervals(const planb_addr_t* prefixes, const uint8_t* lengths, const uint16_t* next_hops,
                                size_t n, uint32_t flags, planb_addr_t* starts, uint16_t* next_hops_out, size_t cap)
{
    clear_error();
    if (n > 0 && (!prefixes || !lengths || !next_hops)) return fail(PLANB_EINVAL, "NULL input array with n > 0");
    Intervals iv;
    std::string err;
    int rc;
    try {
        rc = make_intervals(reinterpret_cast<const U128*>(prefixes), lengths, next_hops, n,
                            (flags & PLANB_FLAG_MERGE_EQUAL_NH) != 0, &iv, &err);
    } catch (const std::bad_alloc&) {
        return fail(PLANB_ENOMEM, "out of host memory");
    }
    if (rc != 0) return fail(rc, err);
    const size_t m = iv.starts.size(), w = std::min(m, cap);
    if (starts) std::memcpy(starts, iv.starts.data(), w * sizeof(planb_addr_t));
    if (next_hops_out) std::memcpy(next_hops_out, iv.nh.data(), w * sizeof(uint16_t));
    return (long long)m;
}

long long planb_build_keys(const planb_addr_t* starts, size_t m, uint32_t fanout, planb_addr_t* keys,
                           size_t cap_keys, planb_info_t* info)
{
    clear_error();
    if (m == 0 || !starts) return fail(PLANB_EINVAL, "need m >= 1 interval starts");
    if (fanout != 8 && fanout != 16 && fanout != 32) return fail(PLANB_EINVAL, "fanout must be 8, 16 or 32");
    const U128* s = reinterpret_cast<const U128*>(starts);
    if (s[0] != U128{0, 0}) return fail(PLANB_EINVAL, "starts[0] must be 0");
    for (size_t i = 1; i < m; ++i)
        if (!(s[i - 1] < s[i])) return fail(PLANB_EINVAL, "starts must be strictly increasing");
    Layout lay;
    std::string err;
    int rc = plan_fib_layout(m, fanout, 16, &lay, &err);
    if (rc != 0) return fail(rc == -5 ? PLANB_ERANGE : PLANB_EINVAL, err);
    if (info) layout_to_info(lay, info);
    const size_t slots = lay.total_slots();
    if (!keys || slots > cap_keys) return (long long)slots;
    Intervals iv;
    iv.starts.assign(s, s + m);
    iv.nh.assign(m, 0);
    std::vector<U128> k;
    try {
        fill_keys(iv, lay, 16, &k);
    } catch (const std::bad_alloc&) {
        return fail(PLANB_ENOMEM, "out of host memory");
    }
    std::memcpy(keys, k.data(), slots * sizeof(planb_addr_t));
    return (long long)slots;
}

long long planb_build_image(const planb_addr_t* starts, const uint16_t* next_hops, size_t m, uint32_t fanout,
                            uint32_t key_bits, void* image, size_t cap_bytes, planb_info_t* info)
{
    clear_error();
    if (m == 0 || !starts || !next_hops) return fail(PLANB_EINVAL, "need m >= 1 interval starts and next hops");
    if (m >= (1ull << 31)) return fail(PLANB_ERANGE, "too many intervals (at most 2^31 - 1)");
    if (fanout != 8 && fanout != 16 && fanout != 32) return fail(PLANB_EINVAL, "fanout must be 8, 16 or 32");
    const U128* s = reinterpret_cast<const U128*>(starts);
    if (s[0] != U128{0, 0}) return fail(PLANB_EINVAL, "starts[0] must be 0");
    for (size_t i = 1; i < m; ++i)
        if (!(s[i - 1] < s[i])) return fail(PLANB_EINVAL, "starts must be strictly increasing");
    Intervals iv;
    int kb = 16, rc;
    std::vector<uint8_t> img;
    try {
        iv.starts.assign(s, s + m);
        iv.nh.assign(next_hops, next_hops + m);
        if ((rc = choose_key_bytes(iv, key_bits, &kb)) != PLANB_OK) return rc;
        Layout lay;
        std::string err;
        if ((rc = plan_fib_layout(m, fanout, kb, &lay, &err)) != 0) return fail(rc == -5 ? PLANB_ERANGE : PLANB_EINVAL, err);
        if (info) {
            layout_to_info(lay, info);
            info->key_bits = (uint32_t)kb * 8;
            info->key_bytes = lay.total_slots() * kb;
        }
        const size_t bytes = lay.total_slots() * kb;
        if (!image || bytes > cap_bytes) return (long long)bytes;
        build_image(iv, lay, kb, &img);
    } catch (const std::bad_alloc&) {
        return fail(PLANB_ENOMEM, "out of host memory");
    }
    std::memcpy(image, img.data(), img.size());
    return (long long)img.size();
}

int planb_get_info(const planb_fib_t* fib, planb_info_t* info)
{
    if (!fib || !info) return fail(PLANB_EINVAL, "NULL argument");
    layout_to_info(fib->lay, info);
    info->key_bits = fib->key_bytes_per_slot * 8;
    info->key_bytes = fib->key_bytes;
    info->value_bytes = fib->value_bytes;
    return PLANB_OK;
}

int planb_layout(uint64_t m, uint32_t fanout, uint32_t slots, int trimmed, planb_info_t* info)
{
    if (!info) return fail(PLANB_EINVAL, "NULL info");
    Layout lay;
    std::string err;
    int rc = plan_layout(m, fanout, slots, fanout - 1, slots, trimmed != 0, &lay, &err);
    if (rc != 0) return fail(rc == -5 ? PLANB_ERANGE : PLANB_EINVAL, err);
    layout_to_info(lay, info);
    return PLANB_OK;
}

int planb_set_tuning(planb_fib_t* fib, const planb_tuning_t* tuning)
{
    if (!fib || !tuning) return fail(PLANB_EINVAL, "NULL argument");
    int32_t lds = 0;
    LookupTuning lt;
    int rc = validate_tuning(fib, *tuning, &lt, &lds);
    if (rc != PLANB_OK) return rc;
    fib->tune = lt;
    fib->lds_levels = lds;
    refresh_desc(fib);
    return PLANB_OK;
}

int planb_set_size_tunings(planb_fib_t* fib, const uint64_t* min_lookups, const planb_tuning_t* tunings,
                           uint32_t count)
{
    if (!fib || (count && (!min_lookups || !tunings))) return fail(PLANB_EINVAL, "NULL argument");
    std::vector<planb_fib_t::SizeTuning> v;
    for (uint32_t k = 0; k < count; ++k) {
        if (k && min_lookups[k] <= min_lookups[k - 1])
            return fail(PLANB_EINVAL, "min_lookups must be strictly ascending");
        planb_fib_t::SizeTuning s{};
        s.min_lookups = min_lookups[k];
        int rc = validate_tuning(fib, tunings[k], &s.tune, &s.lds_levels);
        if (rc != PLANB_OK) return rc;
        s.desc = make_desc(fib, s.lds_levels);
        v.push_back(s);
    }
    fib->size_tunings.swap(v);
    return PLANB_OK;
}

int planb_get_size_tunings(const planb_fib_t* fib, uint64_t* min_lookups, planb_tuning_t* tunings, uint32_t cap)
{
    if (!fib) return fail(PLANB_EINVAL, "NULL fib");
    const uint32_t n = (uint32_t)fib->size_tunings.size();
    for (uint32_t k = 0; k < n && k < cap; ++k) {
        const auto& s = fib->size_tunings[k];
        if (min_lookups) min_lookups[k] = s.min_lookups;
        if (tunings)
            tunings[k] = planb_tuning_t{(uint32_t)s.tune.kpl, s.lds_levels, (uint32_t)s.tune.R, (uint32_t)s.tune.block,
                                        s.tune.tops ? 2u : s.tune.bin ? 1u : 0u};
    }
    return (int)n;
}

int planb_get_tuning(const planb_fib_t* fib, planb_tuning_t* tuning)
{
    if (!fib || !tuning) return fail(PLANB_EINVAL, "NULL argument");
    tuning->keys_per_lane = (uint32_t)fib->tune.kpl;
    tuning->lds_levels = fib->lds_levels;
    tuning->lookups_per_group = (uint32_t)fib->tune.R;
    tuning->block_threads = (uint32_t)fib->tune.block;
    tuning->lds_search = fib->tune.tops ? 2u : fib->tune.bin ? 1u : 0u;
    return PLANB_OK;
}

}  // extern "C"
