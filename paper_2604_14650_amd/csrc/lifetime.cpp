// Lifetime of a FIB's device memory: freed after the lookups already enqueued
// on it have finished, without blocking the host or any other stream.
//
// Section 3.6 ("Dynamic FIB Update") swaps a rebuilt structure in and frees
// the old one once the lookups in flight on it are done.  On the GPU, every
// entry point that enqueues work reading a FIB records an event on that
// stream after the work (one event per stream, re-recorded on every use).
// planb_free then enqueues, on a library stream, a wait on each of those
// events followed by stream-ordered frees: the host returns at once, and no
// other stream waits for anything.  hipFree is avoided on this path because
// it implies a device-wide synchronisation.
//
// A FIB's device allocations therefore come from the stream-ordered
// allocator (hipMallocAsync on a library allocation stream, synchronised once
// so that the memory is ready for every stream).  Where that allocator is not
// supported the memory comes from hipMalloc and is freed, with hipFree, only
// when a later library call finds the waits complete.
#include <algorithm>
#include <mutex>
#include <vector>

#include "api_internal.hpp"

namespace planb {

UseEvent::~UseEvent()
{
    if (ev) (void)hipEventDestroy(ev);
}

namespace {

struct DeviceStreams {
    hipStream_t alloc = nullptr;  // stream-ordered allocations (never waits on anything)
    hipStream_t free = nullptr;   // waits on use events, then frees
};

std::mutex g_mu;                        // guards everything below
std::vector<DeviceStreams> g_streams;   // by device ordinal
std::vector<void*> g_plain;             // hipMalloc'd pointers (allocator unsupported)

struct Grave {
    int device;
    hipEvent_t marker;                  // recorded on the free stream after the frees
    std::vector<UseRef> held;           // the waited-on events, kept alive until then
    std::vector<void*> plain;           // hipMalloc'd memory to release with hipFree then
};
std::vector<Grave> g_graves;

hipError_t streams_for(int device, DeviceStreams** out)
{
    if ((int)g_streams.size() <= device) g_streams.resize(device + 1);
    DeviceStreams& d = g_streams[device];
    hipError_t e = hipSuccess;
    if (!d.alloc) e = hipStreamCreateWithFlags(&d.alloc, hipStreamNonBlocking);
    if (e == hipSuccess && !d.free) e = hipStreamCreateWithFlags(&d.free, hipStreamNonBlocking);
    *out = &d;
    return e;
}

bool take_plain(void* p)
{
    auto it = std::find(g_plain.begin(), g_plain.end(), p);
    if (it == g_plain.end()) return false;
    g_plain.erase(it);
    return true;
}

// Releases graves whose frees have run; caller holds g_mu.
void reap_locked()
{
    for (size_t k = 0; k < g_graves.size();) {
        Grave& g = g_graves[k];
        if (hipEventQuery(g.marker) != hipSuccess) {
            ++k;
            continue;
        }
        for (void* p : g.plain) (void)hipFree(p);
        (void)hipEventDestroy(g.marker);
        g_graves.erase(g_graves.begin() + (long)k);  // drops the held events
    }
}

}  // namespace

UseRef note_use(UseLog& log, hipStream_t stream)
{
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return nullptr;
    std::lock_guard<std::mutex> lk(log.mu);
    UseRef* slot = nullptr;
    for (auto& u : log.last)
        if (u.first == stream) slot = &u.second;
    if (!slot) {
        auto ev = std::make_shared<UseEvent>();
        if (hipEventCreateWithFlags(&ev->ev, hipEventDisableTiming) != hipSuccess) {
            ev->ev = nullptr;
            return nullptr;
        }
        log.last.emplace_back(stream, ev);
        slot = &log.last.back().second;
    }
    // re-recording is safe for a free already queued behind this event: a
    // stream wait takes the event's state at the time it is enqueued
    if (hipEventRecord((*slot)->ev, stream) != hipSuccess) return nullptr;
    return *slot;
}

void note_shared_use(UseLog& log, hipStream_t stream, const UseRef& ev)
{
    if (!ev) return;
    std::lock_guard<std::mutex> lk(log.mu);
    for (auto& u : log.last)
        if (u.first == stream) {
            u.second = ev;
            return;
        }
    log.last.emplace_back(stream, ev);
}

hipError_t fib_alloc(int device, void** p, size_t bytes)
{
    *p = nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    reap_locked();
    DeviceStreams* ds = nullptr;
    hipError_t e = streams_for(device, &ds);
    if (e != hipSuccess) return e;
    e = hipMallocAsync(p, std::max<size_t>(bytes, 1), ds->alloc);
    if (e == hipErrorNotSupported) {
        (void)hipGetLastError();
        if ((e = hipMalloc(p, std::max<size_t>(bytes, 1))) == hipSuccess) g_plain.push_back(*p);
        return e;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ds->alloc);
    return e;
}

void free_after(UseLog& log, int device, const std::vector<void*>& ptrs)
{
    std::lock_guard<std::mutex> lk(g_mu);
    reap_locked();
    DeviceStreams* ds = nullptr;
    Grave g{device, nullptr, {}, {}};
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != device) (void)hipSetDevice(device);
    bool ordered = streams_for(device, &ds) == hipSuccess;
    if (ordered) {
        std::lock_guard<std::mutex> lu(log.mu);
        for (auto& u : log.last) {
            if (!u.second || !u.second->ev) continue;
            ordered &= hipStreamWaitEvent(ds->free, u.second->ev, 0) == hipSuccess;
            g.held.push_back(u.second);
        }
    }
    if (!ordered) {  // no ordered path: wait for the whole device, then free
        (void)hipDeviceSynchronize();
        for (void* p : ptrs) {
            if (!p) continue;
            (void)take_plain(p);
            (void)hipFree(p);
        }
        if (prev != device) (void)hipSetDevice(prev);
        return;
    }
    for (void* p : ptrs) {
        if (!p) continue;
        if (take_plain(p))
            g.plain.push_back(p);
        else
            (void)hipFreeAsync(p, ds->free);
    }
    if (hipEventCreateWithFlags(&g.marker, hipEventDisableTiming) == hipSuccess &&
        hipEventRecord(g.marker, ds->free) == hipSuccess) {
        g_graves.push_back(std::move(g));
    } else {  // cannot tell when the frees ran: wait for them here
        (void)hipStreamSynchronize(ds->free);
        for (void* p : g.plain) (void)hipFree(p);
        if (g.marker) (void)hipEventDestroy(g.marker);
    }
    if (prev != device) (void)hipSetDevice(prev);
}

void reap_frees()
{
    std::lock_guard<std::mutex> lk(g_mu);
    reap_locked();
}

}  // namespace planb
