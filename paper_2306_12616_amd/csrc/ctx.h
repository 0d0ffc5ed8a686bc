// Handle state and host helpers shared by the host runtime files.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "internal.h"

struct chebdm_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    // matrix workspace: T_1..T_k then R_0..R_{m-1}, each ld x ld
    void* mats = nullptr;
    size_t mats_bytes = 0;
    int64_t lay_n = -1, lay_ld = -1, lay_count = -1;
    size_t lay_elem = 0;
    // small device buffers
    void* small = nullptr;
    size_t small_bytes = 0;
    int64_t small_M = 0;
    chebdm::DevScalars* scal = nullptr;
    double *c = nullptr, *coef = nullptr, *tau = nullptr, *trb = nullptr, *gram = nullptr, *trD = nullptr;
    double *ftab = nullptr, *xtab = nullptr, *w = nullptr, *partial = nullptr;
    // pinned host mirror for read-backs
    chebdm::DevScalars* h_scal = nullptr;
    double* h_trD = nullptr;
    // optional launch timing: HIP events recorded on the handle's stream
    struct Ev {
        hipEvent_t a = nullptr, b = nullptr;
        int kind = 0, products = 0;
        double flop = 0.0, bytes = 0.0;
    };
    bool prof = false;
    std::vector<Ev> ev;
    size_t ev_used = 0;
    // activations of the chemical-potential network
    float* mlp_work = nullptr;
    int64_t mlp_work_floats = 0;
    // captured graphs of the device part of chebdm_mu_search / chebdm_density, replayed while
    // the call's arguments (and so every kernel argument) are unchanged
    struct Replay {
        std::vector<char> key;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        int products = 0;   // matrix products in the captured sequence
    };
    hipStream_t cap = nullptr;   // capture stream
    Replay replay[4];            // mu search with D, mu search without D, density, Lanczos bounds
    // partial accumulators of K-sliced tail tiles of the products, kGemmScratchBytes
    void* gemm_scratch = nullptr;
    // Lanczos bounds workspace (basis, work vectors, partials, tridiagonal)
    double* lz = nullptr;
    int64_t lz_doubles = 0;
};

namespace chebdm {

// Sets the thread-local message of chebdm_last_error and returns code.
int fail(int code, const std::string& msg);

enum { PROF_GEMM = 0, PROF_COMBINE = 1, PROF_GRAM = 2, PROF_SEARCH = 3 };
// Timed region on the handle's stream (no-op unless profiling is on).
int prof_begin(chebdm_handle h, int kind, int products, double flop, double bytes, size_t* idx);
int prof_end(chebdm_handle h, size_t idx);
// Algorithmic flops of one symmetric n x n product: n^2 (n + 1).
double sym_product_flop(int64_t n);
// Looks up (once per device; the device must be current) the address of the fixed scratch array
// of chebdm_bounds_noalloc.
int noalloc_setup(int device);

}  // namespace chebdm

#define HIP_TRY(expr)                                                                                  \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return ::chebdm::fail(CHEBDM_ERR_HIP, std::string(#expr) + " failed: " + hipGetErrorString(e_)); \
    } while (0)

#define CHECK(call)              \
    do {                         \
        int rc_ = (call);        \
        if (rc_ < 0) return rc_; \
    } while (0)
