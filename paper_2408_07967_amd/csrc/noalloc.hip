// Fixed device scratch of fgs_render_noalloc (for callers that cannot
// allocate device memory): one array per GPU in the library's code object,
// placed when the code object is loaded on a device and kept until the
// process ends.  In host code the array's name is not a device address: the
// address of each device's copy is taken here, once per device with that
// device current (fgs_create calls noalloc_scratch), and only that address
// is handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fgs.h"
#include "fgs_internal.hpp"

static __device__ __align__(256) unsigned char scratch[FGS_NOALLOC_SCRATCH_BYTES];

namespace fgs {

namespace {
constexpr int kNoAllocDevices = 64;
std::mutex g_mu;
unsigned char *g_base[kNoAllocDevices] = {};
}  // namespace

hipError_t noalloc_scratch(int device, unsigned char **base) {
    *base = nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    const bool cached = device >= 0 && device < kNoAllocDevices;
    if (cached && g_base[device]) {
        *base = g_base[device];
        return hipSuccess;
    }
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    if (cached) g_base[device] = static_cast<unsigned char *>(p);
    *base = static_cast<unsigned char *>(p);
    return hipSuccess;
}

}  // namespace fgs
