// Internal definition of the FIB handle and helpers shared by the C-ABI files.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/planb.h"
#include "builder.hpp"
#include "device.hpp"
#include "lookup.hpp"

namespace planb {
struct LearnedModel;  // learned position model state (learned.hip)

// An event recorded after the latest work on one stream that reads an object.
struct UseEvent {
    hipEvent_t ev = nullptr;
    ~UseEvent();
};
using UseRef = std::shared_ptr<UseEvent>;

// Per object (a FIB, a table set): one event per stream that has enqueued
// work reading it, re-recorded on each use (lifetime.cpp).
struct UseLog {
    std::mutex mu;
    std::vector<std::pair<hipStream_t, UseRef>> last;
};

// Records, on `stream`, the end of the work just enqueued there for `log`'s
// object.  Nothing is recorded while the stream is being captured into a
// graph (such work is the graph owner's to order).  Returns the event, or
// null when none was recorded.
UseRef note_use(UseLog& log, hipStream_t stream);
// Makes `ev` (recorded by another object's note_use) the latest use on stream.
void note_shared_use(UseLog& log, hipStream_t stream, const UseRef& ev);
// Device memory owned by a FIB or its model (stream-ordered allocator).
hipError_t fib_alloc(int device, void** p, size_t bytes);
// Frees ptrs (from fib_alloc) once every use recorded in `log` so far has
// completed; returns at once and blocks no stream.
void free_after(UseLog& log, int device, const std::vector<void*>& ptrs);
// Releases bookkeeping of frees that have run.
void reap_frees();
}  // namespace planb

struct planb_fib {
    planb::Intervals iv;   // host copy of the elementary intervals
    planb::Layout lay;     // tree shape
    void* d_keys = nullptr;
    uint16_t* d_vals = nullptr;
    size_t key_bytes = 0, value_bytes = 0;
    int device = 0;
    uint32_t key_bytes_per_slot = 16;  // 16 (128-bit keys) or 8 (hi word only)
    planb::LookupTuning tune;
    int32_t lds_levels = 0;
    planb::TreeDesc desc{};
    planb::LearnedModel* learned = nullptr;
    mutable planb::UseLog uses;  // streams whose enqueued work reads this FIB
    // Launch shapes by call size (planb_set_size_tunings): a call of n lookups
    // uses the last entry with min_lookups <= n, else tune / desc above.
    struct SizeTuning {
        uint64_t min_lookups;
        planb::LookupTuning tune;
        int32_t lds_levels;
        planb::TreeDesc desc;
    };
    std::vector<SizeTuning> size_tunings;  // ascending min_lookups
};

namespace planb {

extern thread_local std::string g_err;
void clear_error();
int fail(int code, const std::string& msg);
int fail_hip(hipError_t e, const char* what);
int check_current_device(const planb_fib_t* fib);
void refresh_desc(planb_fib_t* f);
// The tree descriptor of f with its top lds_levels levels staged in LDS.
TreeDesc make_desc(const planb_fib_t* f, int32_t lds_levels);
// Checks a public tuning against f (sets the error); out / lds_out receive it.
int validate_tuning(const planb_fib_t* f, const planb_tuning_t& tu, LookupTuning* out, int32_t* lds_out);
// Launch shape and descriptor for a call of n lookups.
void shape_for(const planb_fib_t* f, uint64_t n, const LookupTuning** tu, const TreeDesc** desc);
void release_learned(planb_fib_t* f);  // frees the learned model, if any
// Default launch shape (params' keys per lane / LDS levels, if set) and descriptor.
int finish_fib(planb_fib_t* f, const planb_params_t& p);
// Key slot width (4, 8 or 16) for starts whose low words are all zero
// (lo_zero) and whose low 96 bits are all zero (low96_zero); key_bits as in
// planb_params_t.  Sets the error on failure.
int choose_key_bytes(bool lo_zero, bool low96_zero, uint32_t key_bits, int* key_bytes);
// Layout of a FIB's tree over m intervals with key_bytes-wide slots.
int plan_fib_layout(uint64_t m, uint32_t fanout, int key_bytes, Layout* lay, std::string* err);

}  // namespace planb
