// Commutator check of a density matrix: max_ij |(H D - D H)_ij|.
//
// An exact function of H commutes with H (Sec. II.A builds D from H's own
// eigenvectors), so the size of [H, D] measures how far a computed D is from
// any function of H.  H and D are symmetric, hence
//     (H D - D H)[i][j] = sum_k H[i][k] D[j][k] - sum_k D[i][k] H[j][k],
// a product of row panels in both terms (the layout of the chain products):
// one float64 MFMA accumulator takes the first term and then the second with
// the B fragments negated.  The commutator is antisymmetric, so the tiles on
// and above the diagonal cover every |entry|.  Each work-group folds its tile
// to one maximum and merges it into the result with an integer atomic max on
// the bit pattern (non-negative doubles order like their bits; a NaN, whose
// bits exceed every finite value, survives as the result).
#include "gemm_tile.h"

namespace chebdm {

namespace {

constexpr int kBM = 64, kKU = 4, kFM = 2, kFN = 2;   // 2 x 2 waves of 32 x 32

__global__ void __launch_bounds__(256)
k_commutator(const double* __restrict__ H, const double* __restrict__ D, int64_t n, int64_t ld,
             unsigned long long* __restrict__ out) {
    __shared__ double wmax[4];
    const int T = (int)(ld / kBM);
    int ti, tj;
    upper_tile((int)blockIdx.x, T, ti, tj);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int lr = lane & 15, lq = lane >> 4;
    const int64_t row0 = (int64_t)ti * kBM + wm * 32, col0 = (int64_t)tj * kBM + wn * 32;
    f64x4 acc[kFM][kFN];
#pragma unroll
    for (int f = 0; f < kFM; ++f)
#pragma unroll
        for (int q = 0; q < kFN; ++q) acc[f][q] = f64x4{};
    constexpr int CH = 4 * kKU;
#pragma unroll 1
    for (int term = 0; term < 2; ++term) {
        const double* A = term == 0 ? H : D;
        const double* B = term == 0 ? D : H;
        const double* pa = A + (row0 + lr) * ld + lq * kKU;
        const double* pb = B + (col0 + lr) * ld + lq * kKU;
        for (int64_t k = 0; k < ld; k += CH) {
            Frag<double, kKU> a[kFM], b[kFN];
#pragma unroll
            for (int f = 0; f < kFM; ++f) load_frag<double, kKU>(a[f], pa + (int64_t)f * 16 * ld + k);
#pragma unroll
            for (int q = 0; q < kFN; ++q) {
                load_frag<double, kKU>(b[q], pb + (int64_t)q * 16 * ld + k);
                if (term == 1)
#pragma unroll
                    for (int s = 0; s < kKU; ++s) b[q].v[s] = -b[q].v[s];
            }
            mma_chunk<P_F64, kKU, kFM, kFN>(acc, a, b);
        }
    }
    // f64 16 x 16 output layout: lane (lr, lq), register r -> row lq + 4 r, column lr
    double m = 0.0;
#pragma unroll
    for (int f = 0; f < kFM; ++f)
#pragma unroll
        for (int q = 0; q < kFN; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = row0 + f * 16 + lq + 4 * r, col = col0 + q * 16 + lr;
                if (row < n && col < n) {
                    const double v = fabs(acc[f][q][r]);
                    m = (v > m || v != v) ? v : m;
                }
            }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(m, off, 64);
        m = (o > m || o != o) ? o : m;
    }
    if (lane == 0) wmax[wave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = wmax[0];
        for (int w = 1; w < 4; ++w) b = (wmax[w] > b || wmax[w] != wmax[w]) ? wmax[w] : b;
        atomicMax(out, (unsigned long long)__double_as_longlong(b));
    }
}

__global__ void k_zero_u64(unsigned long long* p) {
    if (threadIdx.x == 0) *p = 0ull;
}

// dst (ld x ld, zero padding kept) = src (n x n, leading dimension lds)
__global__ void __launch_bounds__(256)
k_pad_copy(const double* __restrict__ src, int64_t lds, int64_t n, double* __restrict__ dst, int64_t ld) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t i = blockIdx.y;
    if (j < n) dst[i * ld + j] = src[i * lds + j];
}

}  // namespace

hipError_t launch_commutator(const double* H, int64_t ldh, const double* D, int64_t ldd, int64_t n, int64_t ld,
                             double* Hw, double* Dw, double* out, hipStream_t st) {
    if (ld % kBM != 0 || ld < n || n < 1 || n > 65535) return hipErrorInvalidValue;
    const dim3 cgrid((unsigned)((n + 255) / 256), (unsigned)n);
    hipLaunchKernelGGL(k_pad_copy, cgrid, dim3(256), 0, st, H, ldh, n, Hw, ld);
    hipLaunchKernelGGL(k_pad_copy, cgrid, dim3(256), 0, st, D, ldd, n, Dw, ld);
    auto* o = reinterpret_cast<unsigned long long*>(out);
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, o);
    const int T = (int)(ld / kBM);
    hipLaunchKernelGGL(k_commutator, dim3((unsigned)(T * (T + 1) / 2)), dim3(256), 0, st, (const double*)Hw,
                       (const double*)Dw, n, ld, o);
    return hipGetLastError();
}

}  // namespace chebdm
