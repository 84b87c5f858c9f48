// dr_static.hip — the library's static device memory: one fault word per
// device that every kernel reports device-detected faults to (besides the
// caller's workspace, when there is one).
//
// In host code the name of a __device__ variable is only a host-side
// stand-in: its device address is looked up once per device, with that
// device current, and only that address is ever passed to kernels or copies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "dr_internal.hpp"

namespace dr {

// DR_DEVFLAG_* bits of faults seen by any kernel of the library on this
// device since the last dr_check_device_error (zero at load).
__device__ __align__(256) uint32_t g_fault_word;

namespace {

constexpr int kMaxDevices = 64;

struct Slot {
    std::once_flag once;
    hipError_t err = hipSuccess;
    DeviceGlobals g{};
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
    s.g.scratch = nullptr;
    s.g.scratch_bytes = 0;
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

}  // namespace dr
