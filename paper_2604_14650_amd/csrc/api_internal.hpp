// Internal definition of the FIB handle and helpers shared by the C-ABI files.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/planb.h"
#include "builder.hpp"
#include "device.hpp"
#include "lookup.hpp"

namespace planb {
struct LearnedModel;  // learned position model state (learned.hip)
}

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
};

namespace planb {

extern thread_local std::string g_err;
void clear_error();
int fail(int code, const std::string& msg);
int fail_hip(hipError_t e, const char* what);
int check_current_device(const planb_fib_t* fib);
void refresh_desc(planb_fib_t* f);
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
