// rapid_noalloc.hip -- the fixed device scratch of rapid_segment_noalloc.
//
// Callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc) segment one image
// with all of the library's scratch in this file-scope array: the job record
// first, then the per-image layout of the ordinary scratch pool.  Each GPU
// that loads the library holds its own copy until the process ends.  Host
// code never uses the array's name as an address (there it is a host-side
// stand-in): the device address of each GPU's copy comes from
// hipGetSymbolAddress, taken once per device at rapid_init with that device
// current, and only that address reaches kernels and copies.
#include <mutex>

#include "rapid_internal.h"

namespace rapid {

static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
char *g_ptr[MAX_DEVICES] = {};
}  // namespace

hipError_t noalloc_scratch(int device, char **out)
{
    if (device < 0 || device >= MAX_DEVICES || !out) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[device]) {
        // the caller has made `device` current
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[device] = static_cast<char *>(p);
    }
    *out = g_ptr[device];
    return hipSuccess;
}

// The job record of a call, stored into the scratch by a kernel (its value
// travels as a kernel argument, so the call needs no host staging buffer).
__global__ void k_store_job(Job j, Job *dst)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = j;
}

hipError_t launch_store_job(const Job &j, Job *dst, hipStream_t stream)
{
    hipLaunchKernelGGL(k_store_job, dim3(1), dim3(64), 0, stream, j, dst);
    return hipGetLastError();
}

}  // namespace rapid
