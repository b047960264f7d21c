// scratch.hip -- the static device scratch area behind nep_spin_eval_noalloc:
// one fixed array per GPU, so that evaluation needs no device allocation.
#include <hip/hip_runtime.h>

#include <mutex>

#include "scratch.h"

namespace nep {

// Each GPU the library runs on holds its own copy of this array until the
// process ends. Host code must not use the array's name as an address: it
// resolves it once per device with hipGetSymbolAddress and passes that.
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

int scratch_area(void **base, size_t *bytes) {
    static std::mutex mu;
    static void *addr[SCRATCH_MAX_DEVICES] = {};
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= SCRATCH_MAX_DEVICES) {
        (void)hipGetLastError();
        return -1;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return -2;
        }
        addr[dev] = p;
    }
    *base = addr[dev];
    *bytes = SCRATCH_BYTES;
    return 0;
}

}  // namespace nep
