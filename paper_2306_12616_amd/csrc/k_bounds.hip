// Spectral bounds, the spectrum map H -> H~, and traces.
//
// Bounds: Gershgorin discs (the paper asks for the lowest and highest
// eigenvalues e_a, e_b, Sec. II.B, without naming a method).  Since H is
// symmetric, the absolute row sums equal the absolute column sums, so each
// thread owns one column and walks down rows: a wavefront reads 512
// contiguous bytes per row (coalesced), and row chunks are split across
// workgroups.  Partial sums land in a [split][column] buffer and one
// workgroup folds them in a fixed order, so the result is deterministic.
#include <cmath>

#include "internal.h"
#include "reduce.h"

namespace chebdm {

namespace {

constexpr int kColsPerBlock = 256;

__global__ void __launch_bounds__(kColsPerBlock)
k_gersh_partial(const double* __restrict__ H, int64_t n, int64_t ldh, int64_t rows_per_split,
                double* __restrict__ partial) {
    const int64_t j = (int64_t)blockIdx.x * kColsPerBlock + threadIdx.x;
    if (j >= n) return;
    const int64_t i0 = (int64_t)blockIdx.y * rows_per_split;
    const int64_t i1 = i0 + rows_per_split < n ? i0 + rows_per_split : n;
    double s = 0.0;
    const double* p = H + i0 * ldh + j;
#pragma unroll 8
    for (int64_t i = i0; i < i1; ++i, p += ldh) {
        const double v = fabs(*p);
        s += (i == j) ? 0.0 : v;
    }
    partial[(int64_t)blockIdx.y * n + j] = s;
}

constexpr int kColThreads = 256;

// Per column j: r_j = sum of the split partials (fixed order), the disc [d - r_j, d + r_j]
// with d = H[j][j]; per work-group: min, max and a non-finite flag, written to out[3][nb].
__global__ void __launch_bounds__(kColThreads)
k_gersh_cols(const double* __restrict__ H, int64_t n, int64_t ldh, const double* __restrict__ partial, int nsplit,
             double* __restrict__ out, int nb) {
    __shared__ double smem[kColThreads / 64];
    const int64_t j = (int64_t)blockIdx.x * kColThreads + threadIdx.x;
    double lo = INFINITY, hi = -INFINITY, bad = 0.0;
    if (j < n) {
        double r = 0.0;
        for (int sp = 0; sp < nsplit; ++sp) r += partial[(int64_t)sp * n + j];
        const double d = H[j * ldh + j];
        if (!isfinite(r) || !isfinite(d)) bad = 1.0;
        lo = d - r;
        hi = d + r;
    }
    bad = block_sum<kColThreads>(bad, smem);
    lo = block_min<kColThreads>(lo, smem);
    hi = block_max<kColThreads>(hi, smem);
    if (threadIdx.x == 0) {
        out[blockIdx.x] = lo;
        out[nb + blockIdx.x] = hi;
        out[2 * nb + blockIdx.x] = bad;
    }
}

constexpr int kFinalThreads = 256;

__global__ void __launch_bounds__(kFinalThreads)
k_gersh_final(const double* __restrict__ part, int nb, DevScalars* s) {
    __shared__ double smem[kFinalThreads / 64];
    double lo = INFINITY, hi = -INFINITY, bad = 0.0;
    for (int b = threadIdx.x; b < nb; b += kFinalThreads) {
        lo = fmin(lo, part[b]);
        hi = fmax(hi, part[nb + b]);
        bad += part[2 * nb + b];
    }
    bad = block_sum<kFinalThreads>(bad, smem);
    lo = block_min<kFinalThreads>(lo, smem);
    hi = block_max<kFinalThreads>(hi, smem);
    if (threadIdx.x == 0) {
        s->emin = lo;
        s->emax = hi;
        s->nonfinite = bad > 0.0 ? 1 : 0;
    }
}

// T_1 = H~ = (H - cen I) / half; only the n x n part is written.
template <typename T>
__global__ void __launch_bounds__(256)
k_shift(const double* __restrict__ H, int64_t n, int64_t ldh, const DevScalars* __restrict__ s,
        T* __restrict__ out, int64_t ldw) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t i = blockIdx.y;
    if (j >= n) return;
    const double cen = s->cen, half = s->half;
    const double h = H[i * ldh + j];
    out[i * ldw + j] = (T)((i == j ? h - cen : h) / half);
}

template <typename T>
__global__ void __launch_bounds__(256)
k_traces(const T* __restrict__ base, int64_t stride, int64_t n, int64_t ld, double* __restrict__ out) {
    __shared__ double smem[4];
    const T* a = base + (int64_t)blockIdx.x * stride;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) acc += (double)a[i * ld + i];
    acc = block_sum<256>(acc, smem);
    if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

// D = value * I on the n x n block (the degenerate spectrum e_a = e_b).
__global__ void __launch_bounds__(256)
k_fill_identity(double* __restrict__ D, int64_t n, int64_t ldd, double value) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t i = blockIdx.y;
    if (j >= n) return;
    D[i * ldd + j] = (i == j) ? value : 0.0;
}

// D = (double) src on the n x n block.
template <typename T>
__global__ void __launch_bounds__(256)
k_copy_out(const T* __restrict__ src, int64_t ld, int64_t n, double* __restrict__ D, int64_t ldd) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t i = blockIdx.y;
    if (j >= n) return;
    D[i * ldd + j] = (double)src[i * ld + j];
}

}  // namespace

hipError_t launch_fill_identity(double* D, int64_t n, int64_t ldd, double value, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_identity, dim3((unsigned)((n + 255) / 256), (unsigned)n), dim3(256), 0, st, D,
                       n, ldd, value);
    return hipGetLastError();
}

hipError_t launch_copy_out(const void* src, int is_f64, int64_t ld, int64_t n, double* D, int64_t ldd,
                           hipStream_t st) {
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)n);
    if (is_f64)
        hipLaunchKernelGGL(k_copy_out<double>, grid, dim3(256), 0, st, (const double*)src, ld, n, D, ldd);
    else
        hipLaunchKernelGGL(k_copy_out<float>, grid, dim3(256), 0, st, (const float*)src, ld, n, D, ldd);
    return hipGetLastError();
}

hipError_t launch_gershgorin(const double* H, int64_t n, int64_t ldh, double* partial,
                             int64_t partial_cap, DevScalars* s, hipStream_t st) {
    const int64_t col_blocks = (n + kColsPerBlock - 1) / kColsPerBlock;
    int64_t nsplit = (2048 + col_blocks - 1) / col_blocks;
    const int64_t max_split = (n + 31) / 32;
    if (nsplit > max_split) nsplit = max_split;
    if (nsplit < 1) nsplit = 1;
    const int64_t nb = (n + kColThreads - 1) / kColThreads;
    while (nsplit > 1 && nsplit * n + 3 * nb > partial_cap) nsplit >>= 1;
    if (nsplit * n + 3 * nb > partial_cap) return hipErrorInvalidValue;
    const int64_t rows_per_split = (n + nsplit - 1) / nsplit;
    nsplit = (n + rows_per_split - 1) / rows_per_split;
    double* part2 = partial + nsplit * n;
    hipLaunchKernelGGL(k_gersh_partial, dim3((unsigned)col_blocks, (unsigned)nsplit), dim3(kColsPerBlock),
                       0, st, H, n, ldh, rows_per_split, partial);
    hipLaunchKernelGGL(k_gersh_cols, dim3((unsigned)nb), dim3(kColThreads), 0, st, H, n, ldh,
                       (const double*)partial, (int)nsplit, part2, (int)nb);
    hipLaunchKernelGGL(k_gersh_final, dim3(1), dim3(kFinalThreads), 0, st, (const double*)part2, (int)nb, s);
    return hipGetLastError();
}

hipError_t launch_shift(const double* H, int64_t n, int64_t ldh, const DevScalars* s, void* T1,
                        int64_t ldw, int prec, hipStream_t st) {
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)n);
    if (prec == CHEBDM_FP64)
        hipLaunchKernelGGL(k_shift<double>, grid, dim3(256), 0, st, H, n, ldh, s, (double*)T1, ldw);
    else
        hipLaunchKernelGGL(k_shift<float>, grid, dim3(256), 0, st, H, n, ldh, s, (float*)T1, ldw);
    return hipGetLastError();
}

hipError_t launch_traces(const void* base, int64_t stride, int count, int64_t n, int64_t ld,
                         int is_f64, double* out, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    if (is_f64)
        hipLaunchKernelGGL(k_traces<double>, dim3(count), dim3(256), 0, st, (const double*)base,
                           stride, n, ld, out);
    else
        hipLaunchKernelGGL(k_traces<float>, dim3(count), dim3(256), 0, st, (const float*)base,
                           stride, n, ld, out);
    return hipGetLastError();
}

hipError_t launch_trace_f64(const double* D, int64_t n, int64_t ld, double* out, hipStream_t st) {
    return launch_traces(D, 0, 1, n, ld, 1, out, st);
}

}  // namespace chebdm
