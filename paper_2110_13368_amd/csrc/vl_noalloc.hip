// vl_noalloc.hip -- the FP64 mass reduction for callers that cannot allocate
// device memory (code under stream capture, serving loops, harnesses that
// forbid allocation).  vl_mass reduces through partial sums in the context's
// workspace; this variant needs no context: its partial sums live in one
// static device array per GPU, `scratch`, of kNoallocMaxVolumes x kMassBlocks
// doubles (128 KiB), held by the library until the process ends.  Every call
// on a GPU uses that GPU's array, so calls that overlap on one GPU (other
// streams, other threads) race.  The kernels are vl_mass's, so the sums are
// bitwise those of vl_mass.
#include <mutex>

#include "vl_internal.h"

namespace vl {

namespace {

static __device__ __align__(256) double scratch[kNoallocMaxVolumes * kMassBlocks];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// The device address of this GPU's array, looked up once per device with the
// device current.  In host code `scratch` names a host-side stand-in, so only
// the looked-up address is ever handed to a kernel.
hipError_t scratch_on(int dev, double **out)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

hipError_t mass_noalloc(const void *field, int is_f64, long long vol, long long vol_stride, int nvols,
                        double *out_dev, hipStream_t st)
{
    if (nvols < 1 || nvols > kNoallocMaxVolumes) return hipErrorInvalidValue;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    double *part = nullptr;
    if ((e = scratch_on(dev, &part)) != hipSuccess) return e;
    for (int q = 0; q < nvols; ++q)
        if ((e = launch_mass(field, is_f64, q * vol_stride, vol, part + (size_t)q * kMassBlocks, out_dev + q, st)) !=
            hipSuccess)
            return e;
    return hipSuccess;
}

}  // namespace vl
