// Gershgorin bounds for callers that cannot allocate device memory (work under
// stream capture, serving loops, harnesses that forbid hipMalloc).
//
// chebdm_bounds keeps its column partials in the handle's small buffers, which
// the handle allocates on first use.  This variant runs the same kernels with
// those partials, and the scalars the final fold writes, in a fixed static
// device array of 8 MiB (every GPU the library runs on holds its own copy until
// the process ends).  Its address comes from hipGetSymbolAddress, once per
// device with that device current, when a handle on the device is created; host
// code only ever uses that address, never the array's name.  Every call on a
// device shares that device's array: calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "ctx.h"
#include "internal.h"

namespace chebdm {

namespace {

// 64 doubles of scalars, then nsplit x n column partials plus 3 x ceil(n / 256) block results
// (at most about 525,000 doubles at n = 65535, so the split is the one chebdm_bounds uses).
constexpr int64_t kNoAllocDoubles = (int64_t)1 << 20;
constexpr int64_t kNoAllocMaxN = 65535;
constexpr int kMaxDevices = 64;

__device__ __align__(256) double scratch[kNoAllocDoubles];

std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The device's address of `scratch`; `device` must be the current device.
int scratch_of(int device, double** out) {
    if (device < 0 || device >= kMaxDevices) return fail(CHEBDM_ERR_ARG, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(CHEBDM_ERR_HIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
        g_scratch_ptr[device] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[device];
    return 0;
}

// out[0] = emin, out[1] = emax, both NaN when H held NaN or Inf.
__global__ void __launch_bounds__(64) k_bounds_out(const DevScalars* __restrict__ s, double* __restrict__ out) {
    if (threadIdx.x != 0) return;
    const bool bad = s->nonfinite != 0;
    out[0] = bad ? (double)NAN : s->emin;
    out[1] = bad ? (double)NAN : s->emax;
}

}  // namespace

int noalloc_setup(int device) {
    double* p = nullptr;
    return scratch_of(device, &p);
}

}  // namespace chebdm

using namespace chebdm;

extern "C" int chebdm_bounds_noalloc(chebdm_handle h, const double* dH, int64_t n, int64_t ldh, double* d_out) {
    if (n < 1 || n > kNoAllocMaxN)
        return fail(CHEBDM_ERR_ARG, "n must be in [1, " + std::to_string(kNoAllocMaxN) +
                                        "] for the fixed 8 MiB scratch of chebdm_bounds_noalloc");
    if (ldh < n) return fail(CHEBDM_ERR_ARG, "leading dimension smaller than n");
    if (!h || !dH || !d_out) return fail(CHEBDM_ERR_ARG, "NULL argument");
    HIP_TRY(hipSetDevice(h->device));
    double* base = nullptr;
    const int rc = scratch_of(h->device, &base);
    if (rc < 0) return rc;
    DevScalars* s = reinterpret_cast<DevScalars*>(base);
    double* partial = base + 64;
    HIP_TRY(launch_gershgorin(dH, n, ldh, partial, kNoAllocDoubles - 64, s, h->stream));
    hipLaunchKernelGGL(k_bounds_out, dim3(1), dim3(64), 0, h->stream, (const DevScalars*)s, d_out);
    HIP_TRY(hipGetLastError());
    return CHEBDM_OK;
}
