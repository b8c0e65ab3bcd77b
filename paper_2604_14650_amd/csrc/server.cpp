// Serving runtime: several FIBs resident on one GPU, admitted against a device
// memory budget, with continuous batching of arriving bursts.
//
// The paper's router forms lookup batches from NIC bursts in a dedicated LPM
// stage and rebuilds a FIB in the background, swapping it in atomically and
// freeing the old one once in-flight lookups finish (Section 3 "Batching",
// "Dynamic FIB Update"; Section 4 "Thread Pipeline").  Here:
//  * submit() queues a burst (table id, host addresses, host output; the
//    addresses are read, and the output written, before its completion);
//  * poll() completes finished launches (results copied to the caller's
//    buffers, completion times recorded) and packs queued bursts -- from any
//    tables -- into the next free launch slot, so bursts that arrive while
//    others run join the next launch and launches on different streams
//    overlap;
//  * a table is built on the device when a burst first needs it, evicting the
//    least recently used idle tables while the budget would be exceeded;
//  * set_table() on a live id builds the new FIB and swaps it in; the old one
//    is freed when the last launch that used it has completed.
// Every launch carries its own copy of the tree (and model) descriptors of
// the tables it serves, written on its stream with its bursts, so a swap or
// an eviction never changes what a launch already enqueued reads; the FIBs
// themselves are freed after the launches recorded on them (planb_free).
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "api_internal.hpp"
#include "learned.hpp"
#include "multi.hpp"

using namespace planb;

namespace {

double now_us()
{
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now().time_since_epoch()).count();
}


// Host threads for the staging copies, started with the server: a launch's
// gather of its bursts into pinned staging is split over them, since one
// core's memcpy (about 10 GB/s) would bound the launch rate far below what
// the PCIe link carries.  run(fn, parts) calls fn(0) on the calling thread and
// fn(1..parts-1) on the workers, and returns when all have finished.
class CopyPool {
   public:
    explicit CopyPool(unsigned workers)
    {
        for (unsigned k = 0; k < workers; ++k) th_.emplace_back([this, k] { loop(k + 1); });
    }
    ~CopyPool()
    {
        {
            std::lock_guard<std::mutex> g(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto& t : th_) t.join();
    }
    unsigned size() const { return (unsigned)th_.size() + 1; }
    void run(const std::function<void(unsigned)>& fn, unsigned parts)
    {
        parts = std::max(1u, std::min(parts, size()));
        if (parts > 1) {
            std::lock_guard<std::mutex> g(mu_);
            fn_ = &fn;
            parts_ = parts;
            left_ = parts - 1;
            ++gen_;
        }
        if (parts > 1) cv_.notify_all();
        fn(0);
        if (parts > 1) {
            std::unique_lock<std::mutex> g(mu_);
            done_cv_.wait(g, [&] { return left_ == 0; });
            fn_ = nullptr;
        }
    }

   private:
    void loop(unsigned part)
    {
        uint64_t seen = 0;
        for (;;) {
            const std::function<void(unsigned)>* fn = nullptr;
            {
                std::unique_lock<std::mutex> g(mu_);
                cv_.wait(g, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
                if (part < parts_) fn = fn_;
            }
            if (!fn) continue;
            (*fn)(part);
            std::lock_guard<std::mutex> g(mu_);
            if (--left_ == 0) done_cv_.notify_one();
        }
    }
    std::vector<std::thread> th_;
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    const std::function<void(unsigned)>* fn_ = nullptr;
    unsigned parts_ = 0, left_ = 0;
    uint64_t gen_ = 0;
    bool stop_ = false;
};

struct Pending {
    int64_t tag;
    uint32_t table;
    uint32_t n;
    const planb_addr_t* addrs;  // the caller's, valid until the completion is returned
    uint16_t* out;
    double submit_us;
    uint32_t offset = 0;  // position in the launch
};

struct Table {
    bool registered = false;
    std::vector<planb_addr_t> pfx;
    std::vector<uint8_t> len;
    std::vector<uint16_t> nh;
    uint64_t m = 0;              // elementary intervals of the rule set
    planb_fib_t* fib = nullptr;  // resident structure, or NULL
    size_t bytes = 0;
    double last_use = 0;
    int inflight = 0;            // launches in flight that use `fib`
    uint64_t gen = 0;            // bumped whenever `fib` is replaced or evicted
};

// Descriptor area of one launch (host pinned and device copies alike):
// [count u32, pad to 16][BurstRec x max_bursts][TreeDesc x T][ModelDesc x T],
// T = tables one launch may serve; a burst's `table` is its table's index
// among the launch's T descriptors.
struct DescLayout {
    size_t bursts = 16, trees = 0, models = 0, bytes = 0;
    uint32_t max_tables = 0;
    DescLayout() = default;
    DescLayout(uint32_t max_bursts, uint32_t T) : max_tables(T)
    {
        auto up = [](size_t x) { return (x + 15) / 16 * 16; };
        trees = up(bursts + (size_t)max_bursts * sizeof(BurstRec));
        models = up(trees + (size_t)T * sizeof(TreeDesc));
        bytes = up(models + (size_t)T * sizeof(ModelDesc));
    }
};

struct Slot {
    hipStream_t st = nullptr;
    UseRef done;                      // recorded after each launch's results are copied back
    planb_addr_t* h_in = nullptr;
    uint16_t* h_out = nullptr;
    unsigned char* h_desc = nullptr;  // DescLayout
    planb_addr_t* d_in = nullptr;
    uint16_t* d_out = nullptr;
    unsigned char* d_desc = nullptr;
    bool busy = false;
    std::vector<Pending> bursts;
    std::vector<uint32_t> tables;    // tables of the launch
    std::vector<uint64_t> gens;      // their generation when the launch was filled
};

}  // namespace

struct planb_server {
    planb_server_cfg_t cfg{};
    MultiLaunch launch;
    DescLayout lay;
    std::vector<Table> tables;
    std::vector<uint32_t> local;  // table id -> index among the filling launch's tables (or kNone)
    std::deque<Pending> queue;
    std::vector<Slot> slots;
    std::deque<planb_completion_t> done;
    std::vector<std::pair<uintptr_t, uintptr_t>> io;  // registered zero-copy ranges [lo, hi)
    std::unique_ptr<CopyPool> pool;                    // staging copies (not with zero-copy bursts)
    uint64_t used_bytes = 0;
    planb_server_stats_t stats{};
};

namespace {

constexpr uint32_t kNone = 0xFFFFFFFFu;

void server_release(planb_server_t* s)
{
    for (auto& sl : s->slots) {
        if (sl.st) (void)hipStreamSynchronize(sl.st);
        sl.done.reset();
        if (sl.st) (void)hipStreamDestroy(sl.st);
        if (sl.h_in) (void)hipHostFree(sl.h_in);
        if (sl.h_out) (void)hipHostFree(sl.h_out);
        if (sl.h_desc) (void)hipHostFree(sl.h_desc);
        if (sl.d_in) (void)hipFree(sl.d_in);
        if (sl.d_out) (void)hipFree(sl.d_out);
        if (sl.d_desc) (void)hipFree(sl.d_desc);
    }
    for (auto& t : s->tables)
        if (t.fib) planb_free(t.fib);
    delete s;
}

// Device bytes planb_build will allocate for the table (same layout arithmetic).
size_t table_bytes(const Table& t, uint32_t fanout, uint32_t key_bits, bool learned)
{
    const int kb = (int)key_bits / 8;
    Layout lay;
    std::string err;
    if (plan_layout(t.m, fanout, fanout, (uint32_t)leaf_cap_for((int)fanout, kb),
                    (uint32_t)leaf_slots_for((int)fanout, kb), true, &lay, &err) != 0)
        return SIZE_MAX;
    const uint64_t leaves = kb == 8 ? lay.nodes[lay.depth - 1] : 0;
    return lay.total_slots() * kb + (t.m + 63) / 64 * 64 * 2 + (learned ? learned_model_bytes(0, leaves) : 0);
}

// Make table `id` resident; false if the budget cannot be met right now
// (memory held by tables with launches in flight).
int admit(planb_server_t* s, uint32_t id, bool* ok)
{
    Table& t = s->tables[id];
    *ok = true;
    if (t.fib) return PLANB_OK;
    const uint64_t budget = s->cfg.memory_budget;
    const size_t need = table_bytes(t, s->cfg.fanout, s->cfg.key_bits, s->cfg.learned != 0);
    if (budget) {
        if (need > budget) return fail(PLANB_ERANGE, "table " + std::to_string(id) + " alone exceeds the budget");
        while (s->used_bytes + need > budget) {
            int victim = -1;
            for (uint32_t k = 0; k < s->tables.size(); ++k) {
                const Table& c = s->tables[k];
                if (c.fib && c.inflight == 0 && (victim < 0 || c.last_use < s->tables[victim].last_use))
                    victim = (int)k;
            }
            if (victim < 0) {
                *ok = false;
                return PLANB_OK;
            }
            Table& v = s->tables[victim];
            planb_free(v.fib);  // idle: no launch of this server reads it
            s->used_bytes -= v.bytes;
            v.fib = nullptr;
            ++v.gen;
            v.bytes = 0;
            ++s->stats.evictions;
        }
    }
    planb_params_t p{};
    p.fanout = s->cfg.fanout;
    p.key_bits = s->cfg.key_bits;
    planb_fib_t* f = planb_build_ex(t.pfx.data(), t.len.data(), t.nh.data(), t.len.size(), &p);
    if (!f) return planb_last_status() ? planb_last_status() : PLANB_EDEVICE;
    int rc = PLANB_OK;
    planb_train_cfg_t tc{};
    tc.epochs = 8;  // a short run: admission waits for it
    if (s->cfg.learned && (rc = planb_train(f, &tc, nullptr, nullptr)) != PLANB_OK) {
        planb_free(f);
        return rc;
    }
    t.fib = f;
    t.bytes = table_bytes(t, s->cfg.fanout, s->cfg.key_bits, s->cfg.learned != 0);
    s->used_bytes += t.bytes;
    ++s->stats.admissions;
    return PLANB_OK;
}

bool zero_copy(const planb_server_t* s) { return (s->cfg.flags & PLANB_SERVER_ZERO_COPY) != 0; }

void finish_slot(planb_server_t* s, Slot& sl)
{
    const double t = now_us();
    for (Pending& p : sl.bursts) {
        if (!zero_copy(s))  // zero-copy launches wrote the caller's buffer themselves
            std::memcpy(p.out, sl.h_out + p.offset, (size_t)p.n * sizeof(uint16_t));
        planb_completion_t c{};
        c.tag = p.tag;
        c.table = p.table;
        c.n = p.n;
        c.submit_us = p.submit_us;
        c.done_us = t;
        c.status = PLANB_OK;
        s->done.push_back(c);
    }
    for (size_t k = 0; k < sl.tables.size(); ++k) {
        Table& tb = s->tables[sl.tables[k]];
        if (tb.gen == sl.gens[k]) --tb.inflight;  // else replaced meanwhile (and freed after this launch)
    }
    sl.bursts.clear();
    sl.tables.clear();
    sl.gens.clear();
    sl.busy = false;
}

struct CopyJob {
    void* dst;
    const void* src;
    size_t bytes;
};

// Host copies into pinned staging, split over the server's copy threads in
// parts of at least 256 KB.
void run_copies(CopyPool& pool, const std::vector<CopyJob>& jobs, size_t total)
{
    constexpr size_t kPerPart = 256u << 10;
    const unsigned T = (unsigned)std::min<size_t>(pool.size(), std::max<size_t>(1, total / kPerPart));
    auto copy_range = [&](size_t lo, size_t hi) {  // bytes [lo, hi) of the concatenated jobs
        size_t pos = 0;
        for (const CopyJob& j : jobs) {
            const size_t a = std::max(lo, pos), b = std::min(hi, pos + j.bytes);
            if (a < b)
                std::memcpy(static_cast<char*>(j.dst) + (a - pos), static_cast<const char*>(j.src) + (a - pos), b - a);
            pos += j.bytes;
            if (pos >= hi) break;
        }
    };
    const size_t chunk = (total + T - 1) / T;
    pool.run([&](unsigned k) { copy_range(std::min(total, k * chunk), std::min(total, (k + 1) * chunk)); }, T);
}

void complete_with_error(planb_server_t* s, const Pending& p, int status)
{
    planb_completion_t c{};
    c.tag = p.tag;
    c.table = p.table;
    c.n = p.n;
    c.submit_us = p.submit_us;
    c.done_us = now_us();
    c.status = status;
    s->done.push_back(c);
}

// Packs queued bursts into one launch on the slot's stream.  A burst whose
// table cannot be made resident (its rules fail to build, or it alone exceeds
// the budget) completes at once with that error.  Nothing is committed to the
// slot before the launch is enqueued: if enqueueing fails the bursts go back
// to the front of the queue, in order, and the error is returned.
int fill_slot(planb_server_t* s, Slot& sl, bool* launched)
{
    *launched = false;
    const uint32_t maxb = s->cfg.max_bursts, maxl = s->cfg.max_lookups, maxt = s->lay.max_tables;
    uint32_t nb = 0, na = 0;
    BurstRec* desc = reinterpret_cast<BurstRec*>(sl.h_desc + s->lay.bursts);
    std::vector<char> blocked(s->tables.size(), 0);
    std::vector<CopyJob> copies;
    std::vector<Pending> taken;
    std::vector<uint32_t> tabs;
    std::vector<uint64_t> gens;
    std::vector<planb_fib_t*> fibs;
    auto rollback = [&](int rc) {
        for (auto it = taken.rbegin(); it != taken.rend(); ++it) s->queue.push_front(std::move(*it));
        for (uint32_t id : tabs) {
            --s->tables[id].inflight;
            s->local[id] = kNone;
        }
        return rc;
    };
    for (auto it = s->queue.begin(); it != s->queue.end() && nb < maxb;) {
        Pending& p = *it;
        if (na + p.n > maxl) break;  // submit bounds n by max_lookups, so it fits an empty launch
        if (blocked[p.table]) {
            ++it;
            continue;
        }
        if (s->local[p.table] == kNone && tabs.size() == maxt) break;
        bool ok = true;
        int rc = admit(s, p.table, &ok);
        if (rc != PLANB_OK) {
            complete_with_error(s, p, rc);
            it = s->queue.erase(it);
            continue;
        }
        if (!ok) {  // keep it queued until memory frees up
            blocked[p.table] = 1;
            ++it;
            continue;
        }
        Table& t = s->tables[p.table];
        if (s->local[p.table] == kNone) {
            s->local[p.table] = (uint32_t)tabs.size();
            tabs.push_back(p.table);
            gens.push_back(t.gen);
            fibs.push_back(t.fib);
            ++t.inflight;  // no eviction of this table while the launch is built or runs
        }
        if (zero_copy(s)) {  // registered pinned memory, addressed by the device as it is
            desc[nb] = BurstRec{s->local[p.table], p.n, reinterpret_cast<const u64x2*>(p.addrs), p.out};
        } else {
            copies.push_back(CopyJob{sl.h_in + na, p.addrs, (size_t)p.n * sizeof(planb_addr_t)});
            desc[nb] = BurstRec{s->local[p.table], p.n, reinterpret_cast<const u64x2*>(sl.d_in + na), sl.d_out + na};
        }
        p.offset = na;
        na += p.n;
        ++nb;
        t.last_use = now_us();
        taken.push_back(std::move(p));
        it = s->queue.erase(it);
    }
    if (nb == 0) return rollback(PLANB_OK);
    // this launch's own copy of its tables' descriptors
    TreeDesc* trees = reinterpret_cast<TreeDesc*>(sl.h_desc + s->lay.trees);
    ModelDesc* models = reinterpret_cast<ModelDesc*>(sl.h_desc + s->lay.models);
    for (size_t k = 0; k < tabs.size(); ++k) {
        trees[k] = fibs[k]->desc;
        trees[k].lds_levels = 0;  // the multi-FIB kernels stage no tree levels
        trees[k].lds_slots = 0;
        models[k] = ready_model_desc(fibs[k]);
    }
    if (!copies.empty()) run_copies(*s->pool, copies, (size_t)na * sizeof(planb_addr_t));
    std::memcpy(sl.h_desc, &nb, sizeof(uint32_t));
    const BurstRec* d_bursts = reinterpret_cast<const BurstRec*>(sl.d_desc + s->lay.bursts);
    const TreeDesc* d_trees = reinterpret_cast<const TreeDesc*>(sl.d_desc + s->lay.trees);
    const ModelDesc* d_models = reinterpret_cast<const ModelDesc*>(sl.d_desc + s->lay.models);
    const uint32_t* d_count = reinterpret_cast<const uint32_t*>(sl.d_desc);
    const uint32_t nt = (uint32_t)tabs.size();
    hipError_t e;
    const bool zc = zero_copy(s);
    if ((!zc && (e = hipMemcpyAsync(sl.d_in, sl.h_in, (size_t)na * 16, hipMemcpyHostToDevice, sl.st)) != hipSuccess) ||
        (e = hipMemcpyAsync(sl.d_desc, sl.h_desc, s->lay.bytes, hipMemcpyHostToDevice, sl.st)) != hipSuccess ||
        (e = s->cfg.learned ? launch_multi_learned(s->launch, d_trees, d_models, nt, d_bursts, d_count, maxb, nullptr,
                                                   sl.st)
                            : launch_multi(s->launch, d_trees, nt, d_bursts, d_count, maxb, sl.st)) != hipSuccess ||
        (!zc && (e = hipMemcpyAsync(sl.h_out, sl.d_out, (size_t)na * 2, hipMemcpyDeviceToHost, sl.st)) != hipSuccess) ||
        (e = hipEventRecord(sl.done->ev, sl.st)) != hipSuccess) {
        // work already enqueued on the stream may still read the staging buffers:
        // wait for it before they can be refilled
        (void)hipStreamSynchronize(sl.st);
        return rollback(fail_hip(e, "server launch"));
    }
    for (planb_fib_t* f : fibs) note_shared_use(f->uses, sl.st, sl.done);  // frees wait for this launch
    for (uint32_t id : tabs) s->local[id] = kNone;
    sl.bursts = std::move(taken);
    sl.tables = std::move(tabs);
    sl.gens = std::move(gens);
    sl.busy = true;
    ++s->stats.launches;
    s->stats.bursts += nb;
    s->stats.lookups += na;
    *launched = true;
    return PLANB_OK;
}

}  // namespace

extern "C" {

double planb_server_now_us(void) { return now_us(); }

planb_server_t* planb_server_create(const planb_server_cfg_t* cfg_in)
{
    clear_error();
    planb_server_cfg_t cfg{};
    if (cfg_in) cfg = *cfg_in;
    if (cfg.max_tables == 0) cfg.max_tables = 16;
    if (cfg.streams == 0) cfg.streams = 2;
    if (cfg.max_bursts == 0) cfg.max_bursts = 1024;
    if (cfg.max_lookups == 0) cfg.max_lookups = 1u << 20;
    if (cfg.fanout == 0) cfg.fanout = 16;
    if (cfg.key_bits == 0) cfg.key_bits = 128;
    if ((cfg.key_bits != 32 && cfg.key_bits != 64 && cfg.key_bits != 128) ||
        (cfg.fanout != 8 && cfg.fanout != 16 && cfg.fanout != 32)) {
        fail(PLANB_EINVAL, "server fanout must be 8/16/32 and key_bits 32, 64 or 128");
        return nullptr;
    }
    if (cfg.streams > 8 || cfg.max_tables > 65536 || cfg.max_bursts > 16384 || cfg.learned > 1 ||
        (cfg.flags & ~PLANB_SERVER_ZERO_COPY)) {
        fail(PLANB_EINVAL, "server configuration out of range");
        return nullptr;
    }
    auto* s = new (std::nothrow) planb_server_t();
    if (!s) {
        fail(PLANB_ENOMEM, "out of host memory");
        return nullptr;
    }
    s->cfg = cfg;
    s->tables.resize(cfg.max_tables);
    s->local.assign(cfg.max_tables, kNone);
    s->lay = DescLayout(cfg.max_bursts, std::min(cfg.max_bursts, cfg.max_tables));
    LookupTuning tu;
    tu.kpl = cfg.fanout >= 16 ? 4 : 2;
    tu.R = 2;
    tu.block = 512;
    const int kb = (int)cfg.key_bits / 8;
    if ((cfg.learned ? plan_multi_learned((int)cfg.fanout, kb, cfg.max_bursts, &s->launch)
                     : plan_multi((int)cfg.fanout, kb, tu, cfg.max_bursts, &s->launch)) != PLANB_OK) {
        server_release(s);
        return nullptr;
    }
    s->slots.resize(cfg.streams);
    const size_t dbytes = s->lay.bytes;
    const bool staged = !zero_copy(s);  // zero-copy launches need no address or output staging
    hipError_t e = hipSuccess;
    for (auto& sl : s->slots) {
        sl.done = std::make_shared<UseEvent>();
        if ((e = hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&sl.done->ev, hipEventDisableTiming)) != hipSuccess ||
            (staged &&
             (e = hipHostMalloc(reinterpret_cast<void**>(&sl.h_in), (size_t)cfg.max_lookups * 16, 0)) != hipSuccess) ||
            (staged &&
             (e = hipHostMalloc(reinterpret_cast<void**>(&sl.h_out), (size_t)cfg.max_lookups * 2, 0)) != hipSuccess) ||
            (e = hipHostMalloc(reinterpret_cast<void**>(&sl.h_desc), dbytes, 0)) != hipSuccess ||
            (staged && (e = hipMalloc(reinterpret_cast<void**>(&sl.d_in), (size_t)cfg.max_lookups * 16)) != hipSuccess) ||
            (staged && (e = hipMalloc(reinterpret_cast<void**>(&sl.d_out), (size_t)cfg.max_lookups * 2)) != hipSuccess) ||
            (e = hipMalloc(reinterpret_cast<void**>(&sl.d_desc), dbytes)) != hipSuccess)
            break;
    }
    if (e == hipSuccess && staged) {
        // up to 8 copying threads in all (the caller's and 7 workers)
        const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
        try {
            s->pool = std::make_unique<CopyPool>(std::min(7u, hw > 1 ? hw - 1 : 0u));
        } catch (...) {
            fail(PLANB_ENOMEM, "cannot start the server's copy threads");
            server_release(s);
            return nullptr;
        }
    }
    if (e != hipSuccess) {
        fail_hip(e, "creating the server");
        server_release(s);
        return nullptr;
    }
    return s;
}

void planb_server_free(planb_server_t* s)
{
    if (s) server_release(s);
}

int planb_server_set_table(planb_server_t* s, uint32_t id, const planb_addr_t* prefixes, const uint8_t* lengths,
                           const uint16_t* next_hops, size_t n)
{
    if (!s) return fail(PLANB_EINVAL, "NULL server");
    if (id >= s->cfg.max_tables) return fail(PLANB_ERANGE, "table id out of range");
    if (n && (!prefixes || !lengths || !next_hops)) return fail(PLANB_EINVAL, "NULL rule array");
    // validate now so that a bad rule set never replaces a good one
    long long m = planb_build_intervals(prefixes, lengths, next_hops, n, 0, nullptr, nullptr, 0);
    if (m < 0) return (int)m;
    Table& t = s->tables[id];
    if (t.fib) {  // rebuild-and-swap: retire the live structure, freed after the launches that read it
        s->used_bytes -= t.bytes;
        planb_free(t.fib);
        t.fib = nullptr;
        t.bytes = 0;
        t.inflight = 0;
        ++t.gen;
    }
    t.registered = true;
    t.m = (uint64_t)m;
    t.pfx.assign(prefixes, prefixes + n);
    t.len.assign(lengths, lengths + n);
    t.nh.assign(next_hops, next_hops + n);
    return PLANB_OK;
}

int planb_server_submit(planb_server_t* s, uint32_t table, const planb_addr_t* addrs, uint32_t n, uint16_t* out,
                        int64_t tag)
{
    if (!s) return fail(PLANB_EINVAL, "NULL server");
    if (table >= s->cfg.max_tables || !s->tables[table].registered) return fail(PLANB_EINVAL, "unknown table id");
    if (n > s->cfg.max_lookups) return fail(PLANB_ERANGE, "burst larger than max_lookups");
    if (n && (!addrs || !out)) return fail(PLANB_EINVAL, "NULL host buffer");
    if (n && zero_copy(s)) {  // the kernels will address both buffers: they must be registered pinned memory
        auto inside = [&](const void* p, size_t bytes) {
            const uintptr_t lo = reinterpret_cast<uintptr_t>(p), hi = lo + bytes;
            for (const auto& r : s->io)
                if (lo >= r.first && hi <= r.second) return true;
            return false;
        };
        if (!inside(addrs, (size_t)n * sizeof(planb_addr_t)) || !inside(out, (size_t)n * sizeof(uint16_t)))
            return fail(PLANB_EINVAL, "zero-copy bursts must lie in memory registered with planb_server_register_io");
        if (reinterpret_cast<uintptr_t>(addrs) % 16 || reinterpret_cast<uintptr_t>(out) % 2)
            return fail(PLANB_EINVAL, "misaligned burst buffer");
    }
    Pending p;
    p.tag = tag;
    p.table = table;
    p.n = n;
    p.addrs = addrs;
    p.out = out;
    p.submit_us = now_us();
    s->queue.push_back(std::move(p));
    return PLANB_OK;
}

int planb_server_register_io(planb_server_t* s, const void* base, size_t bytes)
{
    if (!s || !base || bytes == 0) return fail(PLANB_EINVAL, "NULL server or empty range");
    if (s->io.size() >= 64) return fail(PLANB_ERANGE, "at most 64 I/O ranges");
    // both ends must be pinned host memory that the device addresses as the host does
    for (const char* p : {static_cast<const char*>(base), static_cast<const char*>(base) + bytes - 1}) {
        hipPointerAttribute_t a{};
        hipError_t e = hipPointerGetAttributes(&a, p);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(PLANB_EINVAL, "I/O range is not pinned host memory (hipPointerGetAttributes failed)");
        }
        if (a.type != hipMemoryTypeHost || !a.devicePointer || a.devicePointer != a.hostPointer)
            return fail(PLANB_EINVAL, "I/O range must be pinned host memory addressed by the device as by the host");
    }
    // and one allocation: two adjacent pinned blocks could enclose memory that is not
    void* abase = nullptr;
    size_t asize = 0;
    if (hipMemGetAddressRange(&abase, &asize, const_cast<void*>(base)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(PLANB_EINVAL, "I/O range: the allocation holding it is unknown to the runtime");
    }
    const uintptr_t lo = reinterpret_cast<uintptr_t>(base), alo = reinterpret_cast<uintptr_t>(abase);
    if (lo < alo || lo + bytes > alo + asize) return fail(PLANB_EINVAL, "I/O range spans more than one allocation");
    s->io.emplace_back(lo, lo + bytes);
    return PLANB_OK;
}

int planb_server_poll(planb_server_t* s, planb_completion_t* out, uint32_t cap, int block)
{
    if (!s) return fail(PLANB_EINVAL, "NULL server");
    for (;;) {
        for (auto& sl : s->slots) {
            if (!sl.busy) continue;
            hipError_t q = hipEventQuery(sl.done->ev);
            if (q == hipSuccess) {
                finish_slot(s, sl);
            } else if (q != hipErrorNotReady) {
                return fail_hip(q, "server completion");
            }
        }
        for (auto& sl : s->slots) {
            if (sl.busy || s->queue.empty()) continue;
            bool launched = false;
            int rc = fill_slot(s, sl, &launched);
            if (rc != PLANB_OK) return rc;
            if (!launched) break;
        }
        bool any_busy = false;
        for (auto& sl : s->slots) any_busy |= sl.busy;
        if (!block || !s->done.empty() || (!any_busy && s->queue.empty())) break;
        if (!any_busy && !s->queue.empty())  // queued bursts cannot be admitted and nothing will free memory
            return fail(PLANB_ERANGE, "queued bursts need more memory than the budget allows");
    }
    uint32_t k = 0;
    while (k < cap && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    return (int)k;
}

int planb_server_admit(planb_server_t* s, uint32_t id)
{
    if (!s) return fail(PLANB_EINVAL, "NULL server");
    if (id >= s->cfg.max_tables || !s->tables[id].registered) return fail(PLANB_EINVAL, "unknown table id");
    bool ok = true;
    int rc = admit(s, id, &ok);
    if (rc != PLANB_OK) return rc;
    return ok ? PLANB_OK : fail(PLANB_ERANGE, "no idle table to evict for this one");
}

int planb_server_replay(planb_server_t* s, uint32_t n_bursts, const double* arrival_us, const uint32_t* table,
                        const uint64_t* offsets, const planb_addr_t* addrs, uint16_t* out, double* latency_us,
                        double* wall_s)
{
    if (!s || (n_bursts && (!arrival_us || !table || !offsets || !addrs || !out || !latency_us)))
        return fail(PLANB_EINVAL, "NULL argument");
    for (uint32_t k = 1; k < n_bursts; ++k)
        if (arrival_us[k] < arrival_us[k - 1] || offsets[k] < offsets[k - 1])
            return fail(PLANB_EINVAL, "arrivals and offsets must be non-decreasing");
    std::vector<double> sched(n_bursts);
    const double t0 = now_us() + 1000.0;
    for (uint32_t k = 0; k < n_bursts; ++k) sched[k] = t0 + arrival_us[k];
    std::vector<planb_completion_t> comp(1024);
    uint32_t next = 0, done = 0;
    while (done < n_bursts) {
        const double now = now_us();
        while (next < n_bursts && sched[next] <= now) {
            const uint64_t o = offsets[next];
            int rc = planb_server_submit(s, table[next], addrs + o, (uint32_t)(offsets[next + 1] - o), out + o,
                                         (int64_t)next);
            if (rc != PLANB_OK) return rc;
            ++next;
        }
        const int got = planb_server_poll(s, comp.data(), (uint32_t)comp.size(), 0);
        if (got < 0) return got;
        for (int k = 0; k < got; ++k) {
            const int64_t tag = comp[k].tag;
            latency_us[tag] = comp[k].done_us - sched[tag];
            ++done;
        }
    }
    if (wall_s) *wall_s = (now_us() - t0) / 1e6;
    return PLANB_OK;
}

int planb_server_stats(const planb_server_t* s, planb_server_stats_t* st)
{
    if (!s || !st) return fail(PLANB_EINVAL, "NULL argument");
    *st = s->stats;
    st->resident_bytes = s->used_bytes;
    st->resident_tables = 0;
    for (const auto& t : s->tables) st->resident_tables += t.fib != nullptr;
    st->queued = (uint32_t)s->queue.size();
    return PLANB_OK;
}

}  // extern "C"
