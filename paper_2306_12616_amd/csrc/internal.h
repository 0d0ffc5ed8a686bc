// Internal declarations shared by the kernel files and the host runtime.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "chebdm.h"

namespace chebdm {

// Scalars that live on the device so that a pipeline can run without host
// round trips (bounds -> scaling -> mu -> coefficients).
struct DevScalars {
    double emin, emax;    // spectral bounds
    double cen, half;     // H~ = (H - cen I) / half
    double beta_s;        // beta' = beta * half
    double mu_s;          // mu~ = (mu - cen) / half
    double trace;         // t(mu~) from the bisection, or tr D
    double n_elec;        // target electron count
    double tol;           // bisection tolerance
    double lo, hi;        // final bracket
    int32_t nonfinite;    // H held NaN/Inf
    int32_t status;       // CHEBDM_OK / WARN_NOCONV / ERR_BRACKET
    int32_t iters;        // bisection sweeps
    int32_t max_iter;
    int32_t evals;        // evaluations of t(mu~) in the search (bracket checks included)
    int32_t learned;      // 1: the network's bracket held; 0: plain search (or fallback)
};

constexpr int kMaxGroup = 32;   // GEMMs per grouped launch (one Algorithm-1 stage)
constexpr int kMaxBlocks = 48;  // max k and max m (order <= 48*48 - 1)

// One product of the chain: Out = alpha * A B + beta * C + gamma * E + delta * I.
// A and B are symmetric polynomials of H~ (so A B is symmetric and both
// operands may be read along rows); C, E may be null.
template <typename T>
struct GemmDesc {
    const T* A;
    const T* B;
    const T* C;
    const T* E;
    void* Out;          // T* (workspace) or double* (final D) - see out_f64
    int64_t ld_out;
    double alpha, beta, gamma, delta;
    int32_t out_f64;    // 1: Out is a double matrix (final density), else T
    int32_t pad;
};

template <typename T>
struct GemmBatch {
    GemmDesc<T> d[kMaxGroup];
    int32_t count;
};

// ---- bounds / shift / traces (k_bounds.hip)
hipError_t launch_gershgorin(const double* H, int64_t n, int64_t ldh, double* partial,
                             int64_t partial_cap, DevScalars* s, hipStream_t st);
hipError_t launch_set_scalars(DevScalars* s, double emin, double emax, double beta, double mu,
                              int has_mu, double n_elec, double tol, int max_iter, hipStream_t st,
                              int bounds_on_device = 0);
hipError_t launch_shift(const double* H, int64_t n, int64_t ldh, const DevScalars* s, void* T1,
                        int64_t ldw, int prec, hipStream_t st);
// traces of `count` matrices spaced `stride` elements apart (float or double), into out[0..count)
hipError_t launch_traces(const void* base, int64_t stride, int count, int64_t n, int64_t ld,
                         int is_f64, double* out, hipStream_t st);
hipError_t launch_trace_f64(const double* D, int64_t n, int64_t ld, double* out, hipStream_t st);
hipError_t launch_fill_identity(double* D, int64_t n, int64_t ldd, double value, hipStream_t st);
hipError_t launch_copy_out(const void* src, int is_f64, int64_t ld, int64_t n, double* D, int64_t ldd,
                           hipStream_t st);

// ---- commutator check (k_check.hip): *out = max |H D - D H| (float64 bits written as a double);
// Hw, Dw: ld x ld workspace matrices with zero padding (ld a multiple of 64)
hipError_t launch_commutator(const double* H, int64_t ldh, const double* D, int64_t ldd, int64_t n, int64_t ld,
                             double* Hw, double* Dw, double* out, hipStream_t st);

// ---- Lanczos bounds (k_lanczos.hip)
constexpr int kMaxLanczosSteps = 128;
struct LanczosWork {          // views into one device buffer of lanczos_work_doubles(n, steps) doubles
    double *V, *w, *w2;        // basis v_0..v_{steps-1} (rows of n), work vectors
    double *pa, *pc, *pn;      // per-block partials: alpha, projections, norm
    double *alpha, *beta;      // tridiagonal T (steps each)
    int32_t* state;            // [0]: steps done at a breakdown (0: none), [1]: steps done
};
int64_t lanczos_work_doubles(int64_t n, int steps);
__host__ __device__ LanczosWork lanczos_layout(double* base, int64_t n, int steps);
// Overwrites s->emin / s->emax (which must hold the Gershgorin bounds) with the Lanczos bounds.
// steps in [1, min(n, kMaxLanczosSteps)]; work: lanczos_work_doubles(n, steps) doubles laid out
// by lanczos_layout(work, n, steps).
hipError_t launch_lanczos(const double* H, int64_t n, int64_t ldh, int steps, double margin, uint64_t seed,
                          double* work, DevScalars* s, hipStream_t st);

// ---- coefficients / decomposition / moments / bisection (k_cheb.hip)
hipError_t launch_fermi_coeffs(int order, int M, const DevScalars* s, double* f_tab, double* c_out,
                               hipStream_t st, int damping = 0);
hipError_t launch_block_coeffs(const double* c, int order, int k, int m, int form, double* coef,
                               hipStream_t st);
// composition-form blocks rearranged for two Clenshaw chains split at h (m - h <= h)
hipError_t launch_split_blocks(double* coef, int k, int m, int h, hipStream_t st);
hipError_t launch_assemble_moments(const double* tr_baby, const double* gram, int k, int m,
                                   int order, int64_t n, double* tau, hipStream_t st);
hipError_t launch_dct3(const double* tau, int order, int M, double* w, double* x_tab, hipStream_t st,
                       int damping = 0);
// scratch: M doubles of device memory, free during the call (the Fermi table's buffer)
hipError_t launch_bisect(const double* w, const double* x_tab, int M, DevScalars* s, int mode, double* scratch,
                         hipStream_t st);

// ---- block sums and Gram contractions (k_combine.hip)
// R_l = sum_{i<k} coef[l*k + i] T_i for l < m (T_0 = I implicit, T_i = tbase + (i-1)*stride)
template <typename T>
hipError_t launch_combine(const T* tbase, int64_t stride, int k, int m, const double* coef,
                          T* rbase, int64_t n, int64_t ld, hipStream_t st);
// G[l][i] = <L_l, T_i> (Frobenius) for l < nl, i < nt; L_l, T_i given by pointer lists
template <typename T>
hipError_t launch_gram(const T* const* lmats, int nl, const T* const* tmats, int nt, int64_t nelem,
                       double* partial, int64_t partial_cap, double* G, hipStream_t st);

// ---- matrix products (k_gemm.hip)
// scratch (nullable; kGemmScratchBytes is enough): partial accumulators of the K-sliced tiles
// of a launch's last, nearly empty round, or the pieces of stream-K launches (without scratch the launch
// runs unsplit)
constexpr size_t kGemmScratchBytes = (size_t)64 << 20;
hipError_t launch_gemm_f64(const GemmBatch<double>& b, int64_t n, int64_t ld, hipStream_t st,
                           void* scratch = nullptr, size_t scratch_bytes = 0);
// split: 0 float32 MFMA, 1 bf16x3, 2 bf16x6
hipError_t launch_gemm_f32(const GemmBatch<float>& b, int64_t n, int64_t ld, int split, hipStream_t st,
                           void* scratch = nullptr, size_t scratch_bytes = 0);

}  // namespace chebdm

// ======================================================================
// Batched (many uneven-n problems) path: plan-time geometry and run-time
// problem table, shared by k_batch.hip and api_batch.hip.
namespace chebdm {

struct BatchProblem {      // filled by the host before every run (caller's pointers)
    const double* H;
    double* D;
    int64_t ldh, ldd;
    double beta, n_elec;
};

struct BatchGeom {         // fixed for a plan
    int64_t n, ld;         // size and leading dimension (multiple of 128) of the workspace matrices
    int64_t off;           // element offset of the problem's slot 0 in the batch workspace
    int64_t col_off;       // offset of the problem's column sums in the bounds scratch
    int32_t tile;          // product tile edge: 64, 48 or 32 (chosen by the tuner per size bucket)
    int32_t ntile;         // ceil(n / tile)
};

// Lanczos bounds of a batch (k_lanczos.hip): problem p uses tab[p].H / ldh, geo[p].n, s[p] and
// the workspace base + p * stride (stride >= lanczos_work_doubles(nmax, steps)), laid out by
// lanczos_layout(.., n_p, min(steps, n_p)).  With tab == nullptr: one problem (H, n, ldh).
struct LanczosRun {
    const BatchProblem* tab;
    const BatchGeom* geo;
    const double* H;
    int64_t n, ldh;
    DevScalars* s;
    double* base;
    int64_t stride, nmax;
    int32_t steps, pad;
    double margin;
    uint64_t seed;
};
hipError_t launch_lanczos_run(const LanczosRun& r, int count, hipStream_t st);

struct TileItem {          // one tile of one problem's product in a step
    int32_t p;             // problem
    int32_t t;             // linear index in the problem's upper triangle of tiles
};

// Batched product step: every listed tile of descs[p] (one descriptor per problem).
// prec: CHEBDM_FP64 / FP32 / BF16X3 / BF16X6 (descs point to double or float GemmDescs).
hipError_t launch_batch_gemm(int prec, const void* descs, const BatchGeom* geo, const TileItem* items, int nitems,
                             int* counter, int grid, hipStream_t st);
int batch_gemm_grid(int prec);   // resident 64-thread work-groups for the persistent step kernel

struct BatchDims {         // shared sizes of a plan
    int count, order, k, m, lmax;
    int64_t nmax, ldmax, mcap;
    int prec;
    int damping;           // enum chebdm_damping
};
hipError_t launch_batch_zero(int* p, int n, hipStream_t st);
hipError_t launch_batch_bounds(const BatchDims& d, const BatchProblem* tab, const BatchGeom* geo, double* colsum,
                               DevScalars* s, hipStream_t st);
hipError_t launch_batch_setup(const BatchDims& d, const BatchProblem* tab, const BatchGeom* geo, DevScalars* s,
                              int64_t* mq, double tol, int max_iter, hipStream_t st);
hipError_t launch_batch_shift(const BatchDims& d, const BatchProblem* tab, const BatchGeom* geo, const DevScalars* s,
                              void* mats, hipStream_t st);
hipError_t launch_batch_patch(const BatchDims& d, const BatchProblem* tab, void* final_descs, hipStream_t st);
hipError_t launch_batch_moments(const BatchDims& d, const BatchGeom* geo, const void* mats, double* trb,
                                double* partial, int gram_blocks, double* gram, double* tau, hipStream_t st);
hipError_t launch_batch_coeffs(const BatchDims& d, const int64_t* mq, const DevScalars* s, double* ftab, double* c,
                               double* coef, hipStream_t st);
hipError_t launch_batch_combine(const BatchDims& d, const BatchGeom* geo, const double* coef, void* mats,
                                hipStream_t st);
hipError_t launch_batch_finish(const BatchDims& d, const BatchProblem* tab, const BatchGeom* geo, DevScalars* s,
                               double* mu, double* trD, int with_density, hipStream_t st);

}  // namespace chebdm

// ---- learned chemical potential (k_mlp.hip): 64 -> 256 -> 256 -> 1, ReLU, float32
namespace chebdm {
int64_t mlp_nparams();
// work: 4 * B * 256 + 2 * B + 1 floats for backward (2 * B * 256 for forward)
hipError_t launch_mlp_forward(const float* w, const float* X, int Bn, float* y, float* work, hipStream_t st);
hipError_t launch_mlp_backward(const float* w, const float* X, const float* t, int Bn, float* g, float* work,
                               float* loss, hipStream_t st);
hipError_t launch_mlp_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                           float eps, float bc1, float bc2, hipStream_t st);
// batched features for the network (k_batch.hip) and the search modes:
// mode 0 bisection on [-1, 1]; 1 safeguarded Newton on [-1, 1]; 2 network guess mu_hat:
// verify [mu_hat - delta, mu_hat + delta], Newton inside it, else bisection on [-1, 1]
hipError_t launch_batch_features(const BatchDims& d, const BatchGeom* geo, const double* tau, const DevScalars* s,
                                 float* feat, hipStream_t st);
// scratch: count x mcap doubles of device memory, free during the call
hipError_t launch_batch_search(const BatchDims& d, const double* tau, const int64_t* mq, double* w, double* x,
                               DevScalars* s, int mode, const float* mu_hat, double delta, double* scratch,
                               hipStream_t st);
}  // namespace chebdm
