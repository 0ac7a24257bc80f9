// Fixed device scratch for the entry points of libsllg that must not
// allocate device memory (callers under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc).
//
// The scratch is a file-scope device array: every GPU the library runs on
// holds its own copy, at its own address, until the process ends.  Host code
// never passes the array's name to a kernel or a copy (on the host that name
// is a stand-in, not a device address); it looks up each device's address
// once, with that device current, and uses that address from then on.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "kernels.hpp"

namespace sllg {
namespace {

static __device__ __align__(256) double scratch[3 * kNoAllocMaxSites];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;   // device address of `scratch`, per device (null: not looked up yet)

}  // namespace

hipError_t noalloc_scratch(int device, void** ptr, size_t* bytes)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr.empty()) {
        int count = 0;
        const hipError_t e = hipGetDeviceCount(&count);
        if (e != hipSuccess)
            return e;
        g_scratch_ptr.assign((size_t)(count > 0 ? count : 0), nullptr);
    }
    if (device < 0 || (size_t)device >= g_scratch_ptr.size())
        return hipErrorInvalidDevice;
    if (!g_scratch_ptr[(size_t)device]) {
        int current = 0;
        hipError_t e = hipGetDevice(&current);
        if (e != hipSuccess)
            return e;
        if (current != device && (e = hipSetDevice(device)) != hipSuccess)
            return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (current != device)
            (void)hipSetDevice(current);
        if (e != hipSuccess)
            return e;
        if (!p)
            return hipErrorInvalidSymbol;
        g_scratch_ptr[(size_t)device] = p;
    }
    *ptr = g_scratch_ptr[(size_t)device];
    *bytes = sizeof(scratch);
    return hipSuccess;
}

}  // namespace sllg
