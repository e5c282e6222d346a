// The no-allocation entry point: split_dft_exec with the two-pass
// intermediate held in a static device array instead of a workspace, for
// callers that cannot allocate device memory.
#include "../../include/split_dft.h"
#include "internal.h"

#include <hip/hip_runtime.h>

#include <mutex>

namespace {
constexpr size_t kScratchBytes = SPLIT_DFT_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
static_assert(kScratchBytes % 256 == 0, "whole 256-byte lines");
}  // namespace

// Both planes of a chunk's two-pass intermediate.  Every GPU the library runs
// on holds its own copy until the process ends.  In host code this name is a
// host-side stand-in, not a device address: host code only ever uses the
// per-device address that hipGetSymbolAddress returns (g_addr below).
static __device__ __align__(256) float scratch[kScratchBytes / sizeof(float)];

namespace {

std::mutex g_mu;
float* g_addr[kMaxDevices];  // device address of `scratch` per HIP device, once looked up

// Look the array up on `device`, which the callers have made sure is the
// current device.
hipError_t scratch_address(int device, float** ptr, size_t* bytes)
{
    if (device < 0 || device >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        g_addr[device] = static_cast<float*>(p);
    }
    *ptr = g_addr[device];
    *bytes = kScratchBytes;
    return hipSuccess;
}

}  // namespace

void splitdft::prepare_noalloc_scratch(int device)
{
    float* p = nullptr;
    size_t b = 0;
    (void)scratch_address(device, &p, &b);
}

extern "C" split_dft_status split_dft_exec_noalloc(split_dft_plan_t plan, const float* xr, const float* xi,
                                                   float* yr, float* yi, void* stream)
{
    return splitdft::exec_in_scratch(plan, xr, xi, yr, yi, stream, &scratch_address);
}
