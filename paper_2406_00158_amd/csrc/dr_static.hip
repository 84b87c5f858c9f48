// dr_static.hip — the library's static device memory: one fault word per
// device that every kernel reports device-detected faults to (besides the
// caller's workspace, when there is one), and the scratch area of the
// inclusive scan that allocates nothing (dr_inclusive_scan_noalloc).
//
// In host code the name of a __device__ variable is only a host-side
// stand-in: its device address is looked up once per device, with that
// device current, and only that address is ever passed to kernels or copies.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdio>
#include <mutex>
#include <string>

#include "dr.h"
#include "dr_internal.hpp"

namespace dr {

// DR_DEVFLAG_* bits of faults seen by any kernel of the library on this
// device since the last dr_check_device_error (zero at load).
__device__ __align__(256) uint32_t g_fault_word;

// Workspace of dr_inclusive_scan_noalloc: every call on a device shares it.
constexpr size_t kScratchBytes = (size_t)8 << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

struct Slot {
    std::once_flag once;
    hipError_t err = hipSuccess;
    DeviceGlobals g{};
    std::atomic<bool> scratch_zeroed{false};
};

Slot g_slots[kMaxDevices];

// With `dev` current: the device addresses of the static variables.
void lookup(int dev, Slot& s) {
    int prev = -1;
    s.err = hipGetDevice(&prev);
    if (s.err != hipSuccess) return;
    if (prev != dev && (s.err = hipSetDevice(dev)) != hipSuccess) return;
    void* f = nullptr;
    s.err = hipGetSymbolAddress(&f, HIP_SYMBOL(g_fault_word));
    if (s.err == hipSuccess && f == nullptr) s.err = hipErrorInvalidSymbol;
    s.g.fault = (uint32_t*)f;
    void* sc = nullptr;
    if (s.err == hipSuccess) s.err = hipGetSymbolAddress(&sc, HIP_SYMBOL(scratch));
    if (s.err == hipSuccess && sc == nullptr) s.err = hipErrorInvalidSymbol;
    s.g.scratch = (uint8_t*)sc;
    s.g.scratch_bytes = kScratchBytes;
    s.g.device = dev;
    if (prev != dev) {
        const hipError_t e = hipSetDevice(prev);
        if (s.err == hipSuccess) s.err = e;
    }
}

}  // namespace

hipError_t device_globals(hipStream_t stream, DeviceGlobals& g) {
    int dev = -1;
    hipError_t e = stream ? hipStreamGetDevice(stream, &dev) : hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    Slot& s = g_slots[dev];
    std::call_once(s.once, [&] { lookup(dev, s); });
    if (s.err != hipSuccess) return s.err;
    g = s.g;
    return hipSuccess;
}

// The device's scratch area, zero-filled (by a fill kernel on `stream`,
// ahead of the caller's work) the first time a call uses it.
static hipError_t scratch_for(hipStream_t stream, DeviceGlobals& g) {
    hipError_t e = device_globals(stream, g);
    if (e != hipSuccess) return e;
    Slot& s = g_slots[g.device];
    if (!s.scratch_zeroed.exchange(true)) {
        e = launch_zero(g.scratch, g.scratch_bytes, stream);
        if (e != hipSuccess) s.scratch_zeroed.store(false);
    }
    return e;
}

}  // namespace dr

extern "C" dr_status dr_inclusive_scan_noalloc(const dr_table* table, const dr_view* view, int32_t out_dtype,
                                               uint32_t flags, const dr_tuning* tuning, void* stream) {
    dr::DeviceGlobals g;
    const hipError_t e = dr::scratch_for((hipStream_t)stream, g);
    if (e != hipSuccess) return dr::set_error(DR_ERR_HIP, "static scratch: %s", hipGetErrorString(e));
    dr_status s = DR_OK;
    if (table && table->n_segments > DR_SMALL_TABLE)   // the scratch may hold another table's plan
        s = dr_plan(table, DR_ALGO_SCAN, view, tuning, g.scratch, g.scratch_bytes, stream);
    if (s == DR_OK) s = dr_inclusive_scan(table, view, out_dtype, flags, g.scratch, g.scratch_bytes, tuning, stream);
    if (s == DR_ERR_WORKSPACE) {
        const std::string detail = dr_last_error();
        return dr::set_error(DR_ERR_WORKSPACE,
                             "the call needs more than the %zu bytes of static scratch of "
                             "dr_inclusive_scan_noalloc; use dr_inclusive_scan with a workspace (%s)",
                             g.scratch_bytes, detail.c_str());
    }
    return s;
}
