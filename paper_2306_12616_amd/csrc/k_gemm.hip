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
//   bf16x6  three-way split x = hi + mid + lo; the six products down to 2^-16
//           relative (hh, hm, mh, hl, lh, mm) keep about float32 accuracy.
#include "internal.h"

namespace chebdm {

namespace {

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

enum { P_F64 = 0, P_F32 = 1, P_BF16X3 = 2, P_BF16X6 = 3 };

template <int P> struct Traits;
template <> struct Traits<P_F64> {
    using T = double;
    using Acc = f64x4;
    static constexpr int MK = 1;   // k per MFMA and lane
};
template <> struct Traits<P_F32> {
    using T = float;
    using Acc = f32x4;
    static constexpr int MK = 1;
};
template <> struct Traits<P_BF16X3> {
    using T = float;
    using Acc = f32x4;
    static constexpr int MK = 8;
};
template <> struct Traits<P_BF16X6> {
    using T = float;
    using Acc = f32x4;
    static constexpr int MK = 8;
};

// KU consecutive k of one row per lane, loaded as 16-byte vectors.
template <typename T, int KU>
struct Frag {
    T v[KU];
};

template <typename T, int KU>
__device__ __forceinline__ void load_frag(Frag<T, KU>& f, const T* p) {
    constexpr int PER = 16 / sizeof(T);
    static_assert(KU % PER == 0, "KU must fill 16-byte loads");
#pragma unroll
    for (int c = 0; c < KU / PER; ++c) {
        if constexpr (sizeof(T) == 8) {
            const f64x2 x = *reinterpret_cast<const f64x2*>(p + c * PER);
            f.v[c * 2] = x[0];
            f.v[c * 2 + 1] = x[1];
        } else {
            const f32x4 x = *reinterpret_cast<const f32x4*>(p + c * PER);
#pragma unroll
            for (int t = 0; t < 4; ++t) f.v[c * 4 + t] = x[t];
        }
    }
}

__device__ __forceinline__ void split_bf16(const float* x, bf16x8& hi, bf16x8& lo) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const __bf16 h = (__bf16)x[t];
        hi[t] = h;
        lo[t] = (__bf16)(x[t] - (float)h);
    }
}

__device__ __forceinline__ void split3_bf16(const float* x, bf16x8& hi, bf16x8& mid, bf16x8& lo) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const __bf16 h = (__bf16)x[t];
        const float r = x[t] - (float)h;
        const __bf16 m = (__bf16)r;
        hi[t] = h;
        mid[t] = m;
        lo[t] = (__bf16)(r - (float)m);
    }
}

template <int P, int KU, int FM, int FN>
__device__ __forceinline__ void mma_chunk(typename Traits<P>::Acc (&acc)[FM][FN],
                                          const Frag<typename Traits<P>::T, KU> (&a)[FM],
                                          const Frag<typename Traits<P>::T, KU> (&b)[FN]) {
    if constexpr (P == P_F64) {
#pragma unroll
        for (int s = 0; s < KU; ++s)
#pragma unroll
            for (int f = 0; f < FM; ++f)
#pragma unroll
                for (int g = 0; g < FN; ++g)
                    acc[f][g] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[f].v[s], b[g].v[s], acc[f][g], 0, 0, 0);
    } else if constexpr (P == P_F32) {
#pragma unroll
        for (int s = 0; s < KU; ++s)
#pragma unroll
            for (int f = 0; f < FM; ++f)
#pragma unroll
                for (int g = 0; g < FN; ++g)
                    acc[f][g] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[f].v[s], b[g].v[s], acc[f][g], 0, 0, 0);
    } else if constexpr (P == P_BF16X6) {
        // x = hi + mid + lo; keep every term down to 2^-16 relative, smallest first
#pragma unroll
        for (int s = 0; s < KU / 8; ++s) {
            bf16x8 ah[FM], am[FM], al[FM], bh[FN], bm[FN], bl[FN];
#pragma unroll
            for (int f = 0; f < FM; ++f) split3_bf16(&a[f].v[8 * s], ah[f], am[f], al[f]);
#pragma unroll
            for (int g = 0; g < FN; ++g) split3_bf16(&b[g].v[8 * s], bh[g], bm[g], bl[g]);
#pragma unroll
            for (int f = 0; f < FM; ++f)
#pragma unroll
                for (int g = 0; g < FN; ++g) {
                    acc[f][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[f], bh[g], acc[f][g], 0, 0, 0);
                    acc[f][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[f], bl[g], acc[f][g], 0, 0, 0);
                    acc[f][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[f], bm[g], acc[f][g], 0, 0, 0);
                    acc[f][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[f], bh[g], acc[f][g], 0, 0, 0);
                    acc[f][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[f], bm[g], acc[f][g], 0, 0, 0);
                    acc[f][g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[f], bh[g], acc[f][g], 0, 0, 0);
                }
        }
    } else {
#pragma unroll
        for (int s = 0; s < KU / 8; ++s) {
            bf16x8 ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
            for (int f = 0; f < FM; ++f) split_bf16(&a[f].v[8 * s], ah[f], al[f]);
#pragma unroll
            for (int g = 0; g < FN; ++g) split_bf16(&b[g].v[8 * s], bh[g], bl[g]);
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

// Work-group -> tile order.  Work-groups are dealt round-robin to the 8 XCDs
// (each with its own L2); with XCD = 1 the linear id is permuted so that each
// XCD walks a contiguous stretch of the row-major upper triangle, whose tiles
// share A row panels in that XCD's L2.
template <int XCD>
__device__ __forceinline__ void tile_of_block(int ntri, int& t, int& z) {
    const int gx = gridDim.x;
    int lin = (int)blockIdx.x + (int)blockIdx.z * gx;
    if constexpr (XCD) {
        const int total = gx * (int)gridDim.z;
        const int q = total / 8, r = total % 8;
        const int x = lin % 8, slot = lin / 8;
        lin = x * q + (x < r ? x : r) + slot;
    }
    t = lin % gx;
    z = lin / gx;
    (void)ntri;
}

// BM x BM workgroup tile, WGM x WGN wavefronts, each owning a (BM/WGM) x (BM/WGN) tile
// made of 16 x 16 MFMA blocks; KU consecutive k per lane and chunk (chunk = 4 KU k).
// blockIdx.x enumerates upper-triangle tiles, blockIdx.z the products of a grouped launch.
template <int P, int BM, int WGM, int WGN, int KU, int XCD>
__global__ void __launch_bounds__(64 * WGM * WGN)
k_gemm(const GemmBatch<typename Traits<P>::T> batch, int64_t n, int64_t ld, int64_t kpad, int ntile) {
    using T = typename Traits<P>::T;
    using Acc = typename Traits<P>::Acc;
    constexpr int CH = 4 * KU;                 // k per chunk
    constexpr int WTM = BM / WGM, WTN = BM / WGN;
    constexpr int FM = WTM / 16, FN = WTN / 16;
    static_assert(FM >= 1 && FN >= 1 && WTM % 16 == 0 && WTN % 16 == 0, "wave tile must hold whole MFMA blocks");
    static_assert(KU % Traits<P>::MK == 0, "KU must be a multiple of the MFMA k per lane");

    int tlin, z;
    tile_of_block<XCD>(ntile * (ntile + 1) / 2, tlin, z);
    const GemmDesc<T>& g = batch.d[z];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wm = wave / WGN, wn = wave % WGN;
    int ti, tj;
    upper_tile(tlin, ntile, ti, tj);
    const bool diag_tile = ti == tj;
    const int64_t row0 = (int64_t)ti * BM + wm * WTM;
    const int64_t col0 = (int64_t)tj * BM + wn * WTN;
    const int lr = lane & 15, lq = lane >> 4;

    const T* __restrict__ pa = g.A + (row0 + lr) * ld + lq * KU;
    const T* __restrict__ pb = g.B + (col0 + lr) * ld + lq * KU;

    Acc acc[FM][FN];
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int q = 0; q < FN; ++q) acc[f][q] = Acc{};

    Frag<T, KU> a0[FM], b0[FN], a1[FM], b1[FN];
    auto load = [&](Frag<T, KU>(&fa)[FM], Frag<T, KU>(&fb)[FN], int64_t k) {
#pragma unroll
        for (int f = 0; f < FM; ++f) load_frag<T, KU>(fa[f], pa + (int64_t)f * 16 * ld + k);
#pragma unroll
        for (int q = 0; q < FN; ++q) load_frag<T, KU>(fb[q], pb + (int64_t)q * 16 * ld + k);
    };

    // Two register stages with no branch inside the loop: kpad is a multiple of
    // 2 CH, and the loads past the end are clamped to the last chunks (their
    // values are never used).  Straight-line code lets the compiler wait only
    // for the chunk being consumed while the next one is in flight.
    load(a0, b0, 0);
    load(a1, b1, CH);
    for (int64_t k0 = 0;;) {
        mma_chunk<P, KU, FM, FN>(acc, a0, b0);
        load(a0, b0, (k0 + 2 * CH < kpad) ? k0 + 2 * CH : kpad - 2 * CH);
        mma_chunk<P, KU, FM, FN>(acc, a1, b1);
        load(a1, b1, (k0 + 3 * CH < kpad) ? k0 + 3 * CH : kpad - CH);
        k0 += 2 * CH;
        if (k0 >= kpad) break;
    }

    // Output layout of a 16 x 16 block: lane (lr, lq) holds column lr and, in its
    // r-th register, row 4*lq + r for the f32 and bf16 MFMAs but row lq + 4*r for
    // v_mfma_f64_16x16x4f64 (checked on gfx950).
    //
    // C and E are workspace matrices (ld x ld, zero padded), so every tile
    // position is in bounds: they are read in one unpredicated batch and only
    // the stores are predicated.
    const double alpha = g.alpha, beta = g.beta, gamma = g.gamma, delta = g.delta;
    auto row_of = [&](int f, int r) -> int64_t {
        return row0 + f * 16 + (P == P_F64 ? lq + 4 * r : lq * 4 + r);
    };
    double v[FM][FN][4];
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int q = 0; q < FN; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) v[f][q][r] = alpha * (double)acc[f][q][r];
    if (g.C) {
        const T* __restrict__ C = g.C;
        T cv[FM][FN][4];
#pragma unroll
        for (int f = 0; f < FM; ++f)
#pragma unroll
            for (int q = 0; q < FN; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) cv[f][q][r] = C[row_of(f, r) * ld + col0 + q * 16 + lr];
#pragma unroll
        for (int f = 0; f < FM; ++f)
#pragma unroll
            for (int q = 0; q < FN; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) v[f][q][r] += beta * (double)cv[f][q][r];
    }
    if (g.E) {
        const T* __restrict__ E = g.E;
        T ev[FM][FN][4];
#pragma unroll
        for (int f = 0; f < FM; ++f)
#pragma unroll
            for (int q = 0; q < FN; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) ev[f][q][r] = E[row_of(f, r) * ld + col0 + q * 16 + lr];
#pragma unroll
        for (int f = 0; f < FM; ++f)
#pragma unroll
            for (int q = 0; q < FN; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) v[f][q][r] += gamma * (double)ev[f][q][r];
    }
    const int64_t ldo = g.ld_out;
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int q = 0; q < FN; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = row_of(f, r);
                const int64_t col = col0 + q * 16 + lr;
                if (row < n && col < n && !(diag_tile && row > col)) {
                    const double x = v[f][q][r] + (row == col ? delta : 0.0);
                    const int64_t o = row * ldo + col, om = col * ldo + row;
                    if (g.out_f64) {
                        static_cast<double*>(g.Out)[o] = x;
                        if (row != col) static_cast<double*>(g.Out)[om] = x;
                    } else {
                        static_cast<T*>(g.Out)[o] = (T)x;
                        if (row != col) static_cast<T*>(g.Out)[om] = (T)x;
                    }
                }
            }
}

template <int P, int BM, int WGM, int WGN, int KU, int XCD>
hipError_t launch_cfg(const GemmBatch<typename Traits<P>::T>& b, int64_t n, int64_t ld, hipStream_t st) {
    constexpr int CH = 4 * KU;
    const int64_t kpad = (n + 2 * CH - 1) / (2 * CH) * (2 * CH);
    if (kpad > ld || (n + BM - 1) / BM * BM > ld) return hipErrorInvalidValue;
    const int ntile = (int)((n + BM - 1) / BM);
    dim3 grid((unsigned)(ntile * (ntile + 1) / 2), 1, (unsigned)b.count);
    hipLaunchKernelGGL((k_gemm<P, BM, WGM, WGN, KU, XCD>), grid, dim3(64 * WGM * WGN), 0, st, b, n, ld, kpad,
                       ntile);
    return hipGetLastError();
}

// Configuration from a measured sweep on MI355X (N = 1000/2000/4000): one
// wavefront per 64 x 64 tile (64-thread work-groups, XCD-ordered) is fastest
// whenever the upper triangle offers a few hundred tiles (float64 at N = 4000:
// 59 TFLOP/s algorithmic vs 36 for 2 x 2 waves on 128-tiles); smaller
// problems need more wavefronts per tile to fill the 1024 SIMDs, so they use
// 2 x 2 waves of 32 x 32 on each 64-tile.
template <int P>
hipError_t launch_any(const GemmBatch<typename Traits<P>::T>& b, int64_t n, int64_t ld, hipStream_t st) {
    if (b.count <= 0) return hipSuccess;
    if (b.count > kMaxGroup || ld % 128 != 0) return hipErrorInvalidValue;
    constexpr int KU1 = P == P_F64 ? 4 : (P == P_F32 ? 8 : 16);   // one wave per tile
    constexpr int KU4 = P == P_F64 ? 2 : (P == P_F32 ? 4 : 8);    // four waves per tile
    const int64_t t64 = (n + 63) / 64;
    const int64_t tiles = t64 * (t64 + 1) / 2 * b.count;
    if (tiles >= 400) return launch_cfg<P, 64, 1, 1, KU1, 1>(b, n, ld, st);
    return launch_cfg<P, 64, 2, 2, KU4, 1>(b, n, ld, st);
}

}  // namespace

hipError_t launch_gemm_f64(const GemmBatch<double>& b, int64_t n, int64_t ld, hipStream_t st) {
    return launch_any<P_F64>(b, n, ld, st);
}

hipError_t launch_gemm_f32(const GemmBatch<float>& b, int64_t n, int64_t ld, int split, hipStream_t st) {
    if (split == 2) return launch_any<P_BF16X6>(b, n, ld, st);
    if (split == 1) return launch_any<P_BF16X3>(b, n, ld, st);
    return launch_any<P_F32>(b, n, ld, st);
}

}  // namespace chebdm
