// amber_noalloc.hip -- the device scratch behind amber_init_population_noalloc.
//
// Callers that cannot allocate device memory (code under graph capture,
// serving loops, harnesses that forbid hipMalloc) get a run whose workspace
// is this file-scope device array instead of a caller buffer.  Each GPU the
// library runs on holds its own copy until the process ends.  In host code
// the array's name only stands for it; its device address comes from
// hipGetSymbolAddress, taken once per device with that device current, and
// only that address is ever handed to kernels or copies.
#include <mutex>

#include "amber_internal.h"

namespace amber {

static __device__ __align__(256) uint8_t scratch[NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch(int device, void **ptr)
{
    static std::mutex &mu = *new std::mutex;          // never destroyed
    static void *addr[NOALLOC_MAX_DEVICES] = {};
    if (device < 0 || device >= (int)NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

}  // namespace amber
