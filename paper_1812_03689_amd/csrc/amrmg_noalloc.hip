// amrmg_noalloc.hip -- the device array that amrmg_solve_noalloc carves its
// workspace from, for callers that cannot allocate device memory.
//
// The array lives in the library's code object, so every GPU the library
// runs on holds its own copy, at its own address, from the moment the code
// object is loaded there until the process ends.  In host code the array's
// name is a host-side stand-in, not a device address: host code uses it only
// to look that address up (hipGetSymbolAddress) and then passes the address
// it got, per device, to the kernels like any other workspace.
#include <hip/hip_runtime.h>

#include <mutex>

#include "amrmg_noalloc.hpp"

namespace amrmg {

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
struct Slot {
    bool done = false;
    hipError_t err = hipSuccess;
    void *ptr = nullptr;
};
std::mutex g_mu;
Slot g_slot[NOALLOC_MAX_DEVICES];
}  // namespace

hipError_t noalloc_setup(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    Slot &s = g_slot[device];
    if (s.done) return s.err;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != device) e = hipSetDevice(device);
    void *p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur >= 0 && cur != device) (void)hipSetDevice(cur);
    s.done = true;
    s.err = e;
    s.ptr = e == hipSuccess ? p : nullptr;
    return e;
}

void *noalloc_scratch(int device, hipError_t *err)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) {
        if (err) *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    const Slot &s = g_slot[device];
    if (err) *err = s.done ? s.err : hipErrorNotInitialized;
    return s.done ? s.ptr : nullptr;
}

}  // namespace amrmg
