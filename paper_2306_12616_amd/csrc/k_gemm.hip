// Matrix products of the Chebyshev chain on the MFMA units of gfx950.
//
// Every product here multiplies two polynomials of the same symmetric H~
// (baby steps T_{i+u} = 2 T_i T_u - T_{i-u}, Algorithm 1; the ladder
// T_{(l+1)k} = 2 T_k T_{lk} - T_{(l-1)k}; the giant steps over T_k blocks,
// Sec. II.B / III.B).  Both operands are symmetric, so
//     (A B)[i][j] = sum_k A[i][k] B[j][k]
// and both operands are read along their rows: every lane loads a short
// contiguous k-run (16 bytes) of one row, the layout MFMA wants for its K
// dimension, with no transpose and no LDS staging.  The K order inside a
// chunk is permuted per lane group (lane group q owns k = k0 + q*KU + s),
// which leaves the sum unchanged.
//
// Epilogue (fused, float64 arithmetic): Out = alpha*AB + beta*C + gamma*E + delta*I,
// which covers the three-term update (alpha=2, beta=-1), the Clenshaw step
// R_l + 2 T_k B_{l+1} - B_{l+2}, the Horner step S_j + T_k R, and the "- T_0"
// of the first products (delta = -1) without storing an identity matrix.
//
// Symmetric output: A B is symmetric, so only the tiles on and above the
// diagonal are computed (blockIdx.x enumerates the upper triangle) and every
// value is stored twice, at (i, j) and (j, i); inside a diagonal tile only
// i <= j is kept.  This halves the executed flops and, more importantly,
// keeps every matrix of the chain exactly symmetric: reading B along rows
// equals B only for an exactly symmetric B, and an antisymmetric rounding
// part left in the stored matrices grows along the recurrences (measured:
// 6e-10 in float64 and O(1) in float32 at N = 1000, order 512).
//
// Workspace matrices are ld x ld with ld a multiple of 128 and a zero
// padding outside the leading n x n block; the kernels read whole tiles
// without bounds checks and write only the n x n block, so the padding stays
// zero and contributes nothing along K.
//
// Precisions:
//   f64     v_mfma_f64_16x16x4f64, KU = 2 (one 16-byte double2 per lane and operand)
//   f32     v_mfma_f32_16x16x4f32, KU = 4 (one float4)
//   bf16x3  v_mfma_f32_16x16x32_bf16 on hi/lo splits of float operands:
//           x = hi + lo, hi = bf16(x), lo = bf16(x - hi); AB ~ hi*hi + hi*lo + lo*hi,
//           float32 accumulation (lo*lo, ~2^-16 relative, is dropped).
#include "internal.h"

namespace chebdm {

namespace {

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

enum { P_F64 = 0, P_F32 = 1, P_BF16X3 = 2 };

template <int P> struct Traits;
template <> struct Traits<P_F64> {
    using T = double;
    using Acc = f64x4;
    static constexpr int KU = 2;   // k per lane per chunk
};
template <> struct Traits<P_F32> {
    using T = float;
    using Acc = f32x4;
    static constexpr int KU = 4;
};
template <> struct Traits<P_BF16X3> {
    using T = float;
    using Acc = f32x4;
    static constexpr int KU = 8;
};

template <int P> struct Frag;
template <> struct Frag<P_F64> { f64x2 v; };
template <> struct Frag<P_F32> { f32x4 v; };
template <> struct Frag<P_BF16X3> { f32x4 v0, v1; };

template <int P>
__device__ __forceinline__ void load_frag(Frag<P>& f, const typename Traits<P>::T* p) {
    if constexpr (P == P_F64) {
        f.v = *reinterpret_cast<const f64x2*>(p);
    } else if constexpr (P == P_F32) {
        f.v = *reinterpret_cast<const f32x4*>(p);
    } else {
        f.v0 = *reinterpret_cast<const f32x4*>(p);
        f.v1 = *reinterpret_cast<const f32x4*>(p + 4);
    }
}

__device__ __forceinline__ void split_bf16(const Frag<P_BF16X3>& f, bf16x8& hi, bf16x8& lo) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const float x0 = f.v0[t], x1 = f.v1[t];
        const __bf16 h0 = (__bf16)x0, h1 = (__bf16)x1;
        hi[t] = h0;
        hi[t + 4] = h1;
        lo[t] = (__bf16)(x0 - (float)h0);
        lo[t + 4] = (__bf16)(x1 - (float)h1);
    }
}

template <int P, int FM, int FN>
__device__ __forceinline__ void mma_chunk(typename Traits<P>::Acc (&acc)[FM][FN], const Frag<P> (&a)[FM],
                                          const Frag<P> (&b)[FN]) {
    if constexpr (P == P_F64) {
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int f = 0; f < FM; ++f)
#pragma unroll
                for (int g = 0; g < FN; ++g)
                    acc[f][g] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[f].v[s], b[g].v[s], acc[f][g], 0, 0, 0);
    } else if constexpr (P == P_F32) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int f = 0; f < FM; ++f)
#pragma unroll
                for (int g = 0; g < FN; ++g)
                    acc[f][g] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[f].v[s], b[g].v[s], acc[f][g], 0, 0, 0);
    } else {
        bf16x8 ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
        for (int f = 0; f < FM; ++f) split_bf16(a[f], ah[f], al[f]);
#pragma unroll
        for (int g = 0; g < FN; ++g) split_bf16(b[g], bh[g], bl[g]);
#pragma unroll
        for (int f = 0; f < FM; ++f)
#pragma unroll
            for (int g = 0; g < FN; ++g) {
                acc[f][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[f], bh[g], acc[f][g], 0, 0, 0);
                acc[f][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[f], bl[g], acc[f][g], 0, 0, 0);
                acc[f][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[f], bh[g], acc[f][g], 0, 0, 0);
            }
    }
}

// Tile (I, J), I <= J, of linear index t in the row-major upper triangle of a
// T x T tile grid; row I starts at I*T - I*(I-1)/2.
__device__ __forceinline__ void upper_tile(int t, int T, int& I, int& J) {
    const double b = 2.0 * T + 1.0;
    int i = (int)floor(0.5 * (b - sqrt(b * b - 8.0 * (double)t)));
    if (i < 0) i = 0;
    while (i > 0 && i * T - i * (i - 1) / 2 > t) --i;
    while (i + 1 < T && (i + 1) * T - (i + 1) * i / 2 <= t) ++i;
    I = i;
    J = t - (i * T - i * (i - 1) / 2) + i;
}

// BM x BN workgroup tile, WGM x WGN wavefronts, each owning a (BM/WGM) x (BN/WGN) tile
// made of 16 x 16 MFMA blocks.  blockIdx.x: upper-triangle tile; blockIdx.z: the
// product inside a grouped launch.
template <int P, int BM, int BN, int WGM, int WGN>
__global__ void __launch_bounds__(64 * WGM * WGN)
k_gemm(const GemmBatch<typename Traits<P>::T> batch, int64_t n, int64_t ld, int64_t kpad, int ntile) {
    static_assert(BM == BN, "the symmetric tiling needs square tiles");
    using T = typename Traits<P>::T;
    using Acc = typename Traits<P>::Acc;
    constexpr int KU = Traits<P>::KU;
    constexpr int CH = 4 * KU;                 // k per chunk
    constexpr int WTM = BM / WGM, WTN = BN / WGN;
    constexpr int FM = WTM / 16, FN = WTN / 16;
    static_assert(FM >= 1 && FN >= 1, "wave tile must hold whole MFMA blocks");

    const GemmDesc<T>& g = batch.d[blockIdx.z];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wm = wave / WGN, wn = wave % WGN;
    int ti, tj;
    upper_tile((int)blockIdx.x, ntile, ti, tj);
    const bool diag_tile = ti == tj;
    const int64_t row0 = (int64_t)ti * BM + wm * WTM;
    const int64_t col0 = (int64_t)tj * BN + wn * WTN;
    const int lr = lane & 15, lq = lane >> 4;

    const T* __restrict__ pa = g.A + (row0 + lr) * ld + lq * KU;
    const T* __restrict__ pb = g.B + (col0 + lr) * ld + lq * KU;

    Acc acc[FM][FN];
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int q = 0; q < FN; ++q) acc[f][q] = Acc{};

    Frag<P> a0[FM], b0[FN], a1[FM], b1[FN];
    auto load = [&](Frag<P>(&fa)[FM], Frag<P>(&fb)[FN], int64_t k) {
#pragma unroll
        for (int f = 0; f < FM; ++f) load_frag<P>(fa[f], pa + (int64_t)f * 16 * ld + k);
#pragma unroll
        for (int q = 0; q < FN; ++q) load_frag<P>(fb[q], pb + (int64_t)q * 16 * ld + k);
    };

    // two register stages: the next chunk's loads are in flight while the MFMAs run
    load(a0, b0, 0);
    int64_t k0 = 0;
    while (true) {
        if (k0 + CH < kpad) load(a1, b1, k0 + CH);
        mma_chunk<P, FM, FN>(acc, a0, b0);
        k0 += CH;
        if (k0 >= kpad) break;
        if (k0 + CH < kpad) load(a0, b0, k0 + CH);
        mma_chunk<P, FM, FN>(acc, a1, b1);
        k0 += CH;
        if (k0 >= kpad) break;
    }

    // Output layout of a 16 x 16 block: lane (lr, lq) holds column lr and, in its
    // r-th register, row 4*lq + r for the f32 and bf16 MFMAs but row lq + 4*r for
    // v_mfma_f64_16x16x4f64 (checked on gfx950).
    const double alpha = g.alpha, beta = g.beta, gamma = g.gamma, delta = g.delta;
    const T* __restrict__ C = g.C;
    const T* __restrict__ E = g.E;
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int q = 0; q < FN; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = row0 + f * 16 + (P == P_F64 ? lq + 4 * r : lq * 4 + r);
                const int64_t col = col0 + q * 16 + lr;
                if (row < n && col < n && !(diag_tile && row > col)) {
                    const int64_t idx = row * ld + col;
                    double v = alpha * (double)acc[f][q][r];
                    if (C) v += beta * (double)C[idx];
                    if (E) v += gamma * (double)E[idx];
                    if (row == col) v += delta;
                    const int64_t o = row * g.ld_out + col, om = col * g.ld_out + row;
                    if (g.out_f64) {
                        static_cast<double*>(g.Out)[o] = v;
                        if (row != col) static_cast<double*>(g.Out)[om] = v;
                    } else {
                        static_cast<T*>(g.Out)[o] = (T)v;
                        if (row != col) static_cast<T*>(g.Out)[om] = (T)v;
                    }
                }
            }
}

template <int P, int BM, int BN, int WGM, int WGN>
hipError_t launch_cfg(const GemmBatch<typename Traits<P>::T>& b, int64_t n, int64_t ld,
                      hipStream_t st) {
    constexpr int CH = 4 * Traits<P>::KU;
    const int64_t kpad = (n + CH - 1) / CH * CH;
    if (kpad > ld || (n + BM - 1) / BM * BM > ld || (n + BN - 1) / BN * BN > ld)
        return hipErrorInvalidValue;
    const int ntile = (int)((n + BM - 1) / BM);
    dim3 grid((unsigned)(ntile * (ntile + 1) / 2), 1, (unsigned)b.count);
    hipLaunchKernelGGL((k_gemm<P, BM, BN, WGM, WGN>), grid, dim3(64 * WGM * WGN), 0, st, b, n, ld, kpad,
                       ntile);
    return hipGetLastError();
}

template <int P>
hipError_t launch_any(const GemmBatch<typename Traits<P>::T>& b, int64_t n, int64_t ld, hipStream_t st) {
    if (b.count <= 0) return hipSuccess;
    if (b.count > kMaxGroup || ld % 128 != 0) return hipErrorInvalidValue;
    const int64_t t128 = (n + 127) / 128;
    const int64_t big_tiles = t128 * (t128 + 1) / 2 * b.count;
    if (big_tiles >= 512) return launch_cfg<P, 128, 128, 2, 2>(b, n, ld, st);
    return launch_cfg<P, 64, 64, 2, 2>(b, n, ld, st);
}

}  // namespace

hipError_t launch_gemm_f64(const GemmBatch<double>& b, int64_t n, int64_t ld, hipStream_t st) {
    return launch_any<P_F64>(b, n, ld, st);
}

hipError_t launch_gemm_f32(const GemmBatch<float>& b, int64_t n, int64_t ld, int bf16x3,
                           hipStream_t st) {
    return bf16x3 ? launch_any<P_BF16X3>(b, n, ld, st) : launch_any<P_F32>(b, n, ld, st);
}

}  // namespace chebdm
