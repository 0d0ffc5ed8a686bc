// Block sums and Gram contractions over the stack of Chebyshev matrices.
//
// Combine (Sec. III.B: the block sums S_j = sum_i d_{i,j} T_i are independent
// and can be formed together): all m blocks R_l = sum_{i<k} coef[l][i] T_i
// in one pass over T_1..T_{k-1}, i.e. the skinny product (m x k) (k x N^2).
// The pass is HBM-bound (about 2.9 flop per byte in float64), so each thread
// streams two elements of one row of every T_i once and keeps up to 24 float64
// block accumulators per element in registers (four wavefronts per SIMD in
// both precisions); T_0 = I adds coef[l][0] on the diagonal.
// Full padded rows are processed: the zero padding of T_i yields zero
// padding in R_l, so no column predicate is needed.
//
// Gram: G[l][i] = <L_l, T_i>_F (= tr(L_l T_i) for symmetric matrices), the
// (nl x N^2)(N^2 x nt) contraction behind the trace moments.  It runs on the
// float64 MFMA units with the matrices' elements as the K dimension; float
// matrices are widened to float64 first so the moments keep float64 sums.
// Per-workgroup partials are folded in a fixed order (deterministic).
#include "internal.h"
#include "reduce.h"

namespace chebdm {

namespace {

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

template <typename T> struct Vec;
template <> struct Vec<double> { using V = f64x2; static constexpr int W = 2; };
template <> struct Vec<float> { using V = f32x2; static constexpr int W = 2; };

constexpr int kCombineThreads = 256;

template <typename T, int MB>
__global__ void __launch_bounds__(kCombineThreads)
k_combine(const T* __restrict__ tbase, int64_t stride, int k, int l0, int lcount,
          const double* __restrict__ coef, T* __restrict__ rbase, int64_t n, int64_t ld) {
    using V = typename Vec<T>::V;
    constexpr int W = Vec<T>::W;
    // float32 stages its coefficients in LDS (cs[i][l] = coef[l0 + l][i], zero past lcount) and
    // keeps the next T_i in flight: its loop then reads uniform LDS words instead of one guarded
    // scalar load per block and term (combine bandwidth at n = 1000 / 2000 / 4000: 2.9 / 3.1 /
    // 3.5 -> 4.4 / 3.6 / 4.0 TB/s).  float64 keeps the scalar loads, which measured as fast at
    // n = 4000 and 8 % faster at n = 2000.
    constexpr bool kStage = sizeof(T) == 4;
    const int64_t row = blockIdx.y;
    const int64_t col = ((int64_t)blockIdx.x * kCombineThreads + threadIdx.x) * W;
    const bool live = col < ld;
    const int64_t off = row * ld + (live ? col : 0);
    auto tload = [&](int j) { return *reinterpret_cast<const V*>(tbase + (int64_t)j * stride + off); };
    V t{};
    __shared__ double cs[kStage ? kMaxBlocks : 1][MB];
    if constexpr (kStage) {
        if (k > 1) t = tload(0);   // T_1, in flight while the coefficients are staged
        for (int idx = threadIdx.x; idx < lcount * k; idx += kCombineThreads) {
            const int l = idx / k, i = idx % k;
            cs[i][l] = coef[(int64_t)(l0 + l) * k + i];
        }
        for (int idx = threadIdx.x; idx < (MB - lcount) * k; idx += kCombineThreads)
            cs[idx % k][lcount + idx / k] = 0.0;
        __syncthreads();
    }
    if (!live) return;
    auto coef_at = [&](int i, int l) -> double {
        if constexpr (kStage) return cs[i][l];
        else return l < lcount ? coef[(int64_t)(l0 + l) * k + i] : 0.0;
    };

    double acc[MB][W];
    // T_0 = I: coef[l][0] on the diagonal
#pragma unroll
    for (int l = 0; l < MB; ++l) {
        const double c0 = coef_at(0, l);
#pragma unroll
        for (int w = 0; w < W; ++w) acc[l][w] = (col + w == row) ? c0 : 0.0;
    }
    for (int i = 1; i < k; ++i) {
        V tn{};
        if constexpr (kStage) tn = tload(i < k - 1 ? i : i - 1);   // T_{i+1} (the last step re-reads T_i)
        else t = tload(i - 1);
#pragma unroll
        for (int l = 0; l < MB; ++l) {
            const double c = coef_at(i, l);
#pragma unroll
            for (int w = 0; w < W; ++w) acc[l][w] += c * (double)t[w];
        }
        if constexpr (kStage) t = tn;
    }
#pragma unroll
    for (int l = 0; l < MB; ++l) {
        if (l < lcount) {
            V o;
#pragma unroll
            for (int w = 0; w < W; ++w) o[w] = (T)acc[l][w];
            *reinterpret_cast<V*>(rbase + (int64_t)(l0 + l) * stride + off) = o;
        }
    }
}

template <typename T>
struct PtrList {
    const T* p[kMaxBlocks];
};

constexpr int kGramThreads = 256;
constexpr int kGramMax = 48;   // rows / columns of G handled (3 MFMA blocks of 16)

// VW consecutive elements of one matrix per lane, one 32-byte vector load (4 float64 or 8
// float32), widened to float64 only where the MFMA takes them
template <typename T> struct Raw;
template <> struct Raw<double> { typedef double V __attribute__((ext_vector_type(4))); };
template <> struct Raw<float> { typedef float V __attribute__((ext_vector_type(8))); };

// Chunks of CH = 4 VW consecutive elements: lane group lq holds elements lq VW .. lq VW + VW-1
// of each of its matrices, so every (matrix, chunk) is one whole 128-byte line.
template <typename T, int FM, int FN, int VW = 32 / (int)sizeof(T)>
__global__ void __launch_bounds__(kGramThreads)
k_gram_partial(const PtrList<T> lm, int nl, const PtrList<T> tm, int nt, int64_t nchunk,
               double* __restrict__ partial) {
    using R = typename Raw<T>::V;
    constexpr int CH = 4 * VW;
    __shared__ double red[FM * 16][FN * 16 + 1];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lq = lane >> 4;
    const int64_t gw = (int64_t)blockIdx.x * (kGramThreads / 64) + wave;
    const int64_t nw = (int64_t)gridDim.x * (kGramThreads / 64);
    const int64_t c_begin = nchunk * gw / nw, c_end = nchunk * (gw + 1) / nw;

    const T* pa[FM];
    const T* pb[FN];
#pragma unroll
    for (int f = 0; f < FM; ++f) {
        const int li = f * 16 + lr;
        pa[f] = lm.p[li < nl ? li : 0] + lq * VW;
    }
#pragma unroll
    for (int g = 0; g < FN; ++g) {
        const int ti = g * 16 + lr;
        pb[g] = tm.p[ti < nt ? ti : 0] + lq * VW;
    }
    f64x4 acc[FM][FN];
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int g = 0; g < FN; ++g) acc[f][g] = f64x4{0.0, 0.0, 0.0, 0.0};

    auto load = [&](R (&a)[FM], R (&b)[FN], int64_t c) {
#pragma unroll
        for (int f = 0; f < FM; ++f) a[f] = *reinterpret_cast<const R*>(pa[f] + c * CH);
#pragma unroll
        for (int g = 0; g < FN; ++g) b[g] = *reinterpret_cast<const R*>(pb[g] + c * CH);
    };
    auto mma = [&](const R (&a)[FM], const R (&b)[FN]) {
#pragma unroll
        for (int s = 0; s < VW; ++s)
#pragma unroll
            for (int f = 0; f < FM; ++f)
#pragma unroll
                for (int g = 0; g < FN; ++g)
                    acc[f][g] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a[f][s], (double)b[g][s], acc[f][g],
                                                                    0, 0, 0);
    };
    // two register stages: the next chunk's loads are in flight while a chunk's MFMAs run (the
    // last refill of an even count re-reads its final chunk)
    if (c_begin < c_end) {
        R a0[FM], b0[FN], a1[FM], b1[FN];
        int64_t c = c_begin;
        load(a0, b0, c);
        for (; c + 2 <= c_end; c += 2) {
            load(a1, b1, c + 1);
            mma(a0, b0);
            load(a0, b0, c + 2 < c_end ? c + 2 : c + 1);
            mma(a1, b1);
        }
        if (c < c_end) mma(a0, b0);
    }
    // v_mfma_f64_16x16x4f64 leaves G row 16f + lq + 4r, column 16g + lr in lane (lr, lq),
    // register r; waves add in a fixed order
    for (int w = 0; w < kGramThreads / 64; ++w) {
        if (wave == w) {
#pragma unroll
            for (int f = 0; f < FM; ++f)
#pragma unroll
                for (int g = 0; g < FN; ++g)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        double& slot = red[f * 16 + lq + 4 * r][g * 16 + lr];
                        slot = (w == 0) ? acc[f][g][r] : slot + acc[f][g][r];
                    }
        }
        __syncthreads();
    }
    constexpr int NE = FM * 16 * FN * 16;
    for (int idx = threadIdx.x; idx < NE; idx += kGramThreads) {
        const int rr = idx / (FN * 16), cc = idx % (FN * 16);
        partial[(int64_t)blockIdx.x * kGramMax * kGramMax + rr * kGramMax + cc] = red[rr][cc];
    }
}

// G[l][i] = sum over the blocks' partials: one wavefront per entry, lane j adding blocks
// j, j+64, ... in order, then a fixed butterfly across the lanes (deterministic).
__global__ void __launch_bounds__(256)
k_gram_final(const double* __restrict__ partial, int nblocks, int nl, int nt, double* __restrict__ G) {
    const int idx = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (idx >= nl * nt) return;   // whole wavefronts leave together
    const int l = idx / nt, i = idx % nt;
    double s = 0.0;
    for (int b = lane; b < nblocks; b += 64) s += partial[(int64_t)b * kGramMax * kGramMax + l * kGramMax + i];
    s = wave_sum(s);
    if (lane == 0) G[idx] = s;
}

template <typename T, int FM, int FN>
void launch_gram_fixed(const PtrList<T>& L, int nl, const PtrList<T>& Tm, int nt, int64_t nchunk,
                       int nblocks, double* partial, hipStream_t st) {
    hipLaunchKernelGGL((k_gram_partial<T, FM, FN>), dim3(nblocks), dim3(kGramThreads), 0, st, L, nl, Tm,
                       nt, nchunk, partial);
}

template <typename T, int FM>
void launch_gram_fm(int fn, const PtrList<T>& L, int nl, const PtrList<T>& Tm, int nt, int64_t nchunk,
                    int nblocks, double* partial, hipStream_t st) {
    if (fn == 1) launch_gram_fixed<T, FM, 1>(L, nl, Tm, nt, nchunk, nblocks, partial, st);
    else if (fn == 2) launch_gram_fixed<T, FM, 2>(L, nl, Tm, nt, nchunk, nblocks, partial, st);
    else launch_gram_fixed<T, FM, 3>(L, nl, Tm, nt, nchunk, nblocks, partial, st);
}

}  // namespace

template <typename T>
hipError_t launch_combine(const T* tbase, int64_t stride, int k, int m, const double* coef, T* rbase,
                          int64_t n, int64_t ld, hipStream_t st) {
    constexpr int W = Vec<T>::W;
    if (ld % (W * 2) != 0 || k < 1 || k > kMaxBlocks) return hipErrorInvalidValue;
    const int64_t per_block = (int64_t)kCombineThreads * W;
    dim3 grid((unsigned)((ld + per_block - 1) / per_block), (unsigned)n);
    for (int l0 = 0; l0 < m; l0 += 24) {
        const int cnt = (m - l0) < 24 ? (m - l0) : 24;
        if (cnt <= 8)
            hipLaunchKernelGGL((k_combine<T, 8>), grid, dim3(kCombineThreads), 0, st, tbase, stride, k, l0,
                               cnt, coef, rbase, n, ld);
        else if (cnt <= 16)
            hipLaunchKernelGGL((k_combine<T, 16>), grid, dim3(kCombineThreads), 0, st, tbase, stride, k, l0,
                               cnt, coef, rbase, n, ld);
        else
            hipLaunchKernelGGL((k_combine<T, 24>), grid, dim3(kCombineThreads), 0, st, tbase, stride, k, l0,
                               cnt, coef, rbase, n, ld);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gram(const T* const* lmats, int nl, const T* const* tmats, int nt, int64_t nelem,
                       double* partial, int64_t partial_cap, double* G, hipStream_t st) {
    if (nl <= 0 || nt <= 0) return hipSuccess;
    constexpr int64_t CH = 4 * (32 / (int64_t)sizeof(T));   // elements per chunk
    if (nl > kGramMax || nt > kGramMax || nelem % CH != 0) return hipErrorInvalidValue;
    PtrList<T> L{}, Tm{};
    for (int i = 0; i < nl; ++i) L.p[i] = lmats[i];
    for (int i = 0; i < nt; ++i) Tm.p[i] = tmats[i];
    const int64_t nchunk = nelem / CH;
    int64_t nblocks = 1024;
    if (nblocks * 4 > nchunk) nblocks = (nchunk + 3) / 4;
    if (nblocks < 1) nblocks = 1;
    if (nblocks * kGramMax * kGramMax > partial_cap) nblocks = partial_cap / (kGramMax * kGramMax);
    if (nblocks < 1) return hipErrorInvalidValue;
    const int fm = (nl + 15) / 16, fn = (nt + 15) / 16;
    if (fm == 1) launch_gram_fm<T, 1>(fn, L, nl, Tm, nt, nchunk, (int)nblocks, partial, st);
    else if (fm == 2) launch_gram_fm<T, 2>(fn, L, nl, Tm, nt, nchunk, (int)nblocks, partial, st);
    else launch_gram_fm<T, 3>(fn, L, nl, Tm, nt, nchunk, (int)nblocks, partial, st);
    hipLaunchKernelGGL(k_gram_final, dim3((unsigned)((nl * nt + 3) / 4)), dim3(256), 0, st,
                       (const double*)partial, (int)nblocks, nl, nt, G);
    return hipGetLastError();
}

template hipError_t launch_combine<double>(const double*, int64_t, int, int, const double*, double*, int64_t,
                                           int64_t, hipStream_t);
template hipError_t launch_combine<float>(const float*, int64_t, int, int, const double*, float*, int64_t,
                                          int64_t, hipStream_t);
template hipError_t launch_gram<double>(const double* const*, int, const double* const*, int, int64_t, double*,
                                        int64_t, double*, hipStream_t);
template hipError_t launch_gram<float>(const float* const*, int, const float* const*, int, int64_t, double*,
                                       int64_t, double*, hipStream_t);

}  // namespace chebdm
