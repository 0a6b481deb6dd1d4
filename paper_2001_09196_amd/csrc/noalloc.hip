// Device scratch for the entry points that allocate nothing
// (sn_response_noalloc): a file-scope array of fixed size that every GPU the
// library runs on holds until the process ends.  Host code never uses the
// array's name as an address; it asks the runtime for the array's device
// address once per device (noalloc_scratch) and passes that pointer to the
// kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "sn_kernels.hpp"

namespace sn {

static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};
}  // namespace

// Device address of `scratch` on the current device, looked up with that
// device current on the first call per device and kept; returns the HIP
// error of the lookup (or of hipGetDevice).
hipError_t noalloc_scratch(double** out) {
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace sn
