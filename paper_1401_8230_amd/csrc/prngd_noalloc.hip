// prngd_noalloc.hip -- the fixed device scratch of prngd_fill_noalloc.
//
// prngd_fill_noalloc is for callers that cannot allocate device memory
// (code under graph capture, serving loops, harnesses that forbid it).  Its
// launch state lives in one file-scope device array, `scratch`, which each
// GPU the library runs on holds until the process ends:
//
//   bytes [0, 256)       Control of the look-back kernel (tickets, epoch)
//   bytes [256, 512)     unused
//   bytes [512, end)     tile status words, 8 bytes each
//
// Every call on a GPU shares that GPU's array and finds it as the previous
// call left it, so calls that overlap on one GPU race.  In host code the
// array's name is not a device address: the address comes from
// hipGetSymbolAddress once per device, at set-up, and only that address is
// used afterwards.
#include <hip/hip_runtime.h>

#include <cstring>

#include "prngd_internal.hpp"

namespace prngd {
namespace {

constexpr size_t kScratchBytes = size_t(4) << 20;
constexpr size_t kStatusOffset = 512;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

uint8_t *g_scratch[kMaxDevices] = {};

}  // namespace

size_t noalloc_status_words()
{
    return (kScratchBytes - kStatusOffset) / sizeof(uint64_t);
}

// Set-up of device `dev`, with `dev` current: look up this GPU's copy of
// the array and give its Control the first epoch (the status words start
// zero, which no epoch >= 1 reads as ready).  Idempotent.
hipError_t noalloc_setup(int dev)
{
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    if (g_scratch[dev])
        return hipSuccess;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess)
        return e;
    Control init;
    std::memset(&init, 0, sizeof init);
    init.epoch = 1;
    e = hipMemcpy(ptr, &init, sizeof init, hipMemcpyHostToDevice);
    if (e != hipSuccess)
        return e;
    g_scratch[dev] = static_cast<uint8_t *>(ptr);
    return hipSuccess;
}

// This GPU's scratch: its look-back Control and its status words, or null
// before noalloc_setup(dev).
Control *noalloc_control(int dev)
{
    if (dev < 0 || dev >= kMaxDevices || !g_scratch[dev])
        return nullptr;
    return reinterpret_cast<Control *>(g_scratch[dev]);
}

uint64_t *noalloc_status(int dev)
{
    if (dev < 0 || dev >= kMaxDevices || !g_scratch[dev])
        return nullptr;
    return reinterpret_cast<uint64_t *>(g_scratch[dev] + kStatusOffset);
}

}  // namespace prngd
