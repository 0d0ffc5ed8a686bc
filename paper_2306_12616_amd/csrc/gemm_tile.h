// Tile routine of the symmetric Chebyshev-chain products (shared by the
// single-problem kernel and the batched persistent kernel).  See k_gemm.hip
// for the design; this header only holds device code.
#pragma once

#include <type_traits>

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

// Two floats to a pair of bf16 (round to nearest even, one packed conversion) and those two
// bf16 values back to float, read straight from the packed bits (exact).
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ bf16x2 to_bf16x2(float a, float b, float& ra, float& rb) {
    const bf16x2 h = __builtin_convertvector((f32x2){a, b}, bf16x2);
    const uint32_t u = __builtin_bit_cast(uint32_t, h);
    ra = __builtin_bit_cast(float, u << 16);
    rb = __builtin_bit_cast(float, u & 0xffff0000u);
    return h;
}

// x = hi + lo (+ rounding), hi = bf16(x), lo = bf16(x - hi); pairs of elements share each
// conversion (three VALU operations per element instead of four).
__device__ __forceinline__ void split_bf16(const float* x, bf16x8& hi, bf16x8& lo) {
#pragma unroll
    for (int t = 0; t < 8; t += 2) {
        float h0, h1, u0, u1;
        const bf16x2 h = to_bf16x2(x[t], x[t + 1], h0, h1);
        const bf16x2 l = to_bf16x2(x[t] - h0, x[t + 1] - h1, u0, u1);
        hi[t] = h[0], hi[t + 1] = h[1];
        lo[t] = l[0], lo[t + 1] = l[1];
    }
}

// x = hi + mid + lo (+ rounding): hi = bf16(x), mid = bf16(x - hi), lo = bf16(x - hi - mid).
__device__ __forceinline__ void split3_bf16(const float* x, bf16x8& hi, bf16x8& mid, bf16x8& lo) {
#pragma unroll
    for (int t = 0; t < 8; t += 2) {
        float h0, h1, m0, m1, u0, u1;
        const bf16x2 h = to_bf16x2(x[t], x[t + 1], h0, h1);
        const float r0 = x[t] - h0, r1 = x[t + 1] - h1;
        const bf16x2 m = to_bf16x2(r0, r1, m0, m1);
        const bf16x2 l = to_bf16x2(r0 - m0, r1 - m1, u0, u1);
        hi[t] = h[0], hi[t + 1] = h[1];
        mid[t] = m[0], mid[t + 1] = m[1];
        lo[t] = l[0], lo[t + 1] = l[1];
    }
}

// LOW: the wave tile sits on the diagonal of a diagonal tile (square, row0 == col0), so blocks
// f > g lie wholly below the diagonal, where the epilogue stores nothing: their MFMAs are left out.
template <int P, int KU, int FM, int FN, bool LOW = false>
__device__ __forceinline__ void mma_chunk(typename Traits<P>::Acc (&acc)[FM][FN],
                                          const Frag<typename Traits<P>::T, KU> (&a)[FM],
                                          const Frag<typename Traits<P>::T, KU> (&b)[FN]) {
    static_assert(!LOW || FM == FN, "diagonal blocks of a square wave tile");
    if constexpr (P == P_F64) {
#pragma unroll
        for (int s = 0; s < KU; ++s)
#pragma unroll
            for (int f = 0; f < FM; ++f)
#pragma unroll
                for (int g = 0; g < FN; ++g)
                    if (!LOW || f <= g)
                        acc[f][g] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[f].v[s], b[g].v[s], acc[f][g], 0, 0, 0);
    } else if constexpr (P == P_F32) {
#pragma unroll
        for (int s = 0; s < KU; ++s)
#pragma unroll
            for (int f = 0; f < FM; ++f)
#pragma unroll
                for (int g = 0; g < FN; ++g)
                    if (!LOW || f <= g)
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
                    if (LOW && f > g) continue;
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
                    if (LOW && f > g) continue;
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

// Tile (I, J), I <= J, of linear index t in a blocked order of the upper
// triangle of a T x T tile grid: G x G super-blocks (those on or above the
// diagonal) in row-major order, row-major tiles inside each (the diagonal
// super-blocks hold only their upper triangle).  Consecutive indices then
// cover a compact 2-D region, so tiles that run together on one XCD share
// both their A row panels and their B panels in that XCD's L2.
__device__ __forceinline__ void blocked_tile(int t, int T, int G, int& I, int& J) {
    const int TS = (T + G - 1) / G;
    for (int si = 0; si < TS; ++si) {
        const int rows = T - si * G < G ? T - si * G : G;
        const int diag = rows * (rows + 1) / 2;
        if (t < diag) {
            int i, j;
            upper_tile(t, rows, i, j);
            I = si * G + i;
            J = si * G + j;
            return;
        }
        t -= diag;
        const int rest = rows * (T - (si + 1) * G > 0 ? T - (si + 1) * G : 0);   // super-blocks right of it
        if (t < rest) {
            // the row band's off-diagonal part, ordered super-block by super-block
            for (int sj = si + 1; sj < TS; ++sj) {
                const int cols = T - sj * G < G ? T - sj * G : G;
                if (t < rows * cols) {
                    I = si * G + t / cols;
                    J = sj * G + t % cols;
                    return;
                }
                t -= rows * cols;
            }
        }
        t -= rest;
    }
    I = J = 0;   // not reached for t < T (T + 1) / 2
}

// Epilogue of one wave tile (FM x FN blocks of 16 x 16 at row0, col0):
// Out = alpha*acc + beta*C + gamma*E + delta*I in float64, stored at (i, j) and (j, i).
// RB rows of 16 x 16 blocks are handled per batch: their C and E values are all
// loaded before any is used (RB = FM: one batch for the whole tile; smaller RB
// keeps fewer registers live).
template <int P, int FM, int FN, int RB = FM>
__device__ __forceinline__ void tile_epilogue(const GemmDesc<typename Traits<P>::T>& g,
                                              const typename Traits<P>::Acc (&acc)[FM][FN], int64_t n, int64_t ld,
                                              int64_t row0, int64_t col0, bool diag_tile, int lr, int lq) {
    using T = typename Traits<P>::T;
    static_assert(FM % RB == 0, "row batches must divide the tile");
    // Output layout of a 16 x 16 block: lane (lr, lq) holds column lr and, in its
    // r-th register, row 4*lq + r for the f32 and bf16 MFMAs but row lq + 4*r for
    // v_mfma_f64_16x16x4f64 (checked on gfx950).
    //
    // C and E are workspace matrices (ld x ld, zero padded), so every tile
    // position is in bounds: they are read unpredicated and only the stores are
    // predicated.
    const double alpha = g.alpha, beta = g.beta, gamma = g.gamma, delta = g.delta;
    auto row_of = [&](int f, int r) -> int64_t {
        return row0 + f * 16 + (P == P_F64 ? lq + 4 * r : lq * 4 + r);
    };
    const int64_t ldo = g.ld_out;
#pragma unroll
    for (int f0 = 0; f0 < FM; f0 += RB) {
        double v[RB][FN][4];
#pragma unroll
        for (int f = 0; f < RB; ++f)
#pragma unroll
            for (int q = 0; q < FN; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) v[f][q][r] = alpha * (double)acc[f0 + f][q][r];
        if (g.C) {
            const T* __restrict__ C = g.C;
            T cv[RB][FN][4];
#pragma unroll
            for (int f = 0; f < RB; ++f)
#pragma unroll
                for (int q = 0; q < FN; ++q)
#pragma unroll
                    for (int r = 0; r < 4; ++r) cv[f][q][r] = C[row_of(f0 + f, r) * ld + col0 + q * 16 + lr];
#pragma unroll
            for (int f = 0; f < RB; ++f)
#pragma unroll
                for (int q = 0; q < FN; ++q)
#pragma unroll
                    for (int r = 0; r < 4; ++r) v[f][q][r] += beta * (double)cv[f][q][r];
        }
        if (g.E) {
            const T* __restrict__ E = g.E;
            T ev[RB][FN][4];
#pragma unroll
            for (int f = 0; f < RB; ++f)
#pragma unroll
                for (int q = 0; q < FN; ++q)
#pragma unroll
                    for (int r = 0; r < 4; ++r) ev[f][q][r] = E[row_of(f0 + f, r) * ld + col0 + q * 16 + lr];
#pragma unroll
            for (int f = 0; f < RB; ++f)
#pragma unroll
                for (int q = 0; q < FN; ++q)
#pragma unroll
                    for (int r = 0; r < 4; ++r) v[f][q][r] += gamma * (double)ev[f][q][r];
        }
#pragma unroll
        for (int f = 0; f < RB; ++f)
#pragma unroll
            for (int q = 0; q < FN; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = row_of(f0 + f, r);
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
}

// One BM x BM tile (ti, tj), ti <= tj, of the symmetric product g, computed by
// WGM x WGN x SK wavefronts of the calling work-group: WGM x WGN wave tiles of
// (BM/WGM) x (BM/WGN), each split over SK wavefronts along K (contiguous K
// ranges in units of two chunks) whose partial sums are added through LDS in
// a fixed order (deterministic) before the epilogue.  With SK > 1 the routine
// ends in a work-group barrier, so every thread of the work-group must call it.
// k_lo, k_hi (multiples of 2 CH; k_hi < 0: kpad): the K range of this call.  part != null:
// instead of the epilogue, the work-group's summed accumulators are stored there, lane-native,
// wave tile by wave tile (a K slice of a tile, added up later by gemm_tile_fix).
// SB: instruction order of the K loop.  0: the compiler's; 1: scheduling barriers pin each
// chunk's loads right after the MFMAs of the chunk whose registers they refill, so they are
// in flight while the other chunk's MFMAs run (left alone, the compiler sinks both chunks'
// loads to the end of the loop body, behind most of the MFMAs); -1: 1 for float32 (N = 4000,
// three products: 1.766 -> 1.700 ms; N = 2000, four: 0.425 -> 0.407), 0 otherwise (float64
// already issues them early; no change).
// DS: a wavefront whose wave tile lies on the diagonal of a diagonal tile leaves out the MFMAs of
// the blocks below the diagonal (where dynamic scheduling turns the shorter tile into time saved).
template <int P, int BM, int WGM, int WGN, int KU, int SK = 1, int RB = 16, int SB = -1, bool DS = false>
__device__ __forceinline__ void gemm_tile(const GemmDesc<typename Traits<P>::T>& g, int64_t n, int64_t ld,
                                          int64_t kpad, int ti, int tj, int64_t k_lo = 0, int64_t k_hi = -1,
                                          typename Traits<P>::Acc* part = nullptr) {
    using T = typename Traits<P>::T;
    using Acc = typename Traits<P>::Acc;
    constexpr int CH = 4 * KU;                 // k per chunk
    constexpr int WTM = BM / WGM, WTN = BM / WGN;
    constexpr int FM = WTM / 16, FN = WTN / 16;
    constexpr bool kSB = SB < 0 ? P == P_F32 : SB != 0;
    static_assert(FM >= 1 && FN >= 1 && WTM % 16 == 0 && WTN % 16 == 0, "wave tile must hold whole MFMA blocks");
    static_assert(KU % Traits<P>::MK == 0, "KU must be a multiple of the MFMA k per lane");
    static_assert(SK >= 1 && SK <= 8, "K split of 1..8 wavefronts");

    const int wave_all = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ks = wave_all / (WGM * WGN), wave = wave_all % (WGM * WGN);
    const int wm = wave / WGN, wn = wave % WGN;
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

    // Two register stages: while one chunk's MFMAs run, the other chunk's registers are being
    // refilled.  K ranges come in units of 2 CH; the range that holds the end of K stops at the
    // chunk holding element n - 1 (the rest of kpad is zero padding), so it may hold an odd number
    // of chunks, whose last refill then loads one padding chunk that is not used.  The last one
    // or two chunks are consumed after the loop with no further loads, so the epilogue's addends
    // are the only loads behind them (clamped reloads of the last chunks there cost 1-3 % of the
    // product time, N = 1000 - 4000, and 3 % of the 512-problem batch).
    if (k_hi < 0) k_hi = kpad;
    int64_t kbeg = k_lo, kend = k_hi;
    if constexpr (SK > 1) {
        const int64_t units = (k_hi - k_lo) / (2 * CH);
        kbeg = k_lo + units * ks / SK * (2 * CH);
        kend = k_lo + units * (ks + 1) / SK * (2 * CH);
    }
    // (the split-bf16 tiles keep whole units: their 48-tiles would spill registers with the
    // guarded last chunk)
    constexpr bool kOdd = P == P_F64 || P == P_F32;
    if constexpr (kOdd) {
        const int64_t kceil = (n + CH - 1) / CH * CH;   // kpad or kpad - CH: a non-empty range keeps a chunk
        if (kend > kceil) kend = kceil;
    }
    // One copy of the loop per MFMA set: all blocks, or (DS) the diagonal wave tile's blocks on and
    // above the diagonal.  Every chunk loaded lies below kpad.
    auto kloop = [&](auto low) {
        constexpr bool L = decltype(low)::value;
        load(a0, b0, kbeg);
        load(a1, b1, kbeg + CH);
        int64_t k0 = kbeg;
        for (; k0 + 2 * CH < kend; k0 += 2 * CH) {
            mma_chunk<P, KU, FM, FN, L>(acc, a0, b0);
            if constexpr (kSB) __builtin_amdgcn_sched_barrier(0);
            load(a0, b0, k0 + 2 * CH);
            if constexpr (kSB) __builtin_amdgcn_sched_barrier(0);
            mma_chunk<P, KU, FM, FN, L>(acc, a1, b1);
            if constexpr (kSB) __builtin_amdgcn_sched_barrier(0);
            load(a1, b1, k0 + 3 * CH);
        }
        mma_chunk<P, KU, FM, FN, L>(acc, a0, b0);
        if (!kOdd || k0 + CH < kend) mma_chunk<P, KU, FM, FN, L>(acc, a1, b1);
    };
    if (kend > kbeg) {
        if constexpr (DS && FM == FN) {
            if (diag_tile && row0 == col0) kloop(std::true_type{});
            else kloop(std::false_type{});
        } else {
            kloop(std::false_type{});
        }
    }
    if constexpr (SK > 1) {
        // partial sums of the K slices 1..SK-1 through LDS, added in slice order
        __shared__ Acc red[SK - 1][WGM * WGN][FM * FN][64];
        if (ks > 0) {
#pragma unroll
            for (int f = 0; f < FM; ++f)
#pragma unroll
                for (int q = 0; q < FN; ++q) red[ks - 1][wave][f * FN + q][lane] = acc[f][q];
        }
        __syncthreads();
        if (ks > 0) return;
#pragma unroll
        for (int j = 0; j < SK - 1; ++j)
#pragma unroll
            for (int f = 0; f < FM; ++f)
#pragma unroll
                for (int q = 0; q < FN; ++q) acc[f][q] += red[j][wave][f * FN + q][lane];
    }

    if (part) {
        Acc* dst = part + (int64_t)wave * FM * FN * 64;
#pragma unroll
        for (int f = 0; f < FM; ++f)
#pragma unroll
            for (int q = 0; q < FN; ++q) dst[(f * FN + q) * 64 + lane] = acc[f][q];
        return;
    }
    tile_epilogue<P, FM, FN, (RB < FM ? RB : FM)>(g, acc, n, ld, row0, col0, diag_tile, lr, lq);
}

// Accumulators of one BM x BM tile per K slice (WGM x WGN wave tiles).
template <int P, int BM, int WGM, int WGN>
constexpr int64_t slice_accs() {
    return (int64_t)WGM * WGN * (BM / WGM / 16) * (BM / WGN / 16) * 64;
}

// Sum of the nslice K-slice partials of tile (ti, tj) in slice order, then its epilogue, by the
// WGM x WGN wavefronts of the calling work-group.
template <int P, int BM, int WGM, int WGN, int RB = 16>
__device__ __forceinline__ void gemm_tile_fix(const GemmDesc<typename Traits<P>::T>& g, int64_t n, int64_t ld,
                                              int ti, int tj, const typename Traits<P>::Acc* part, int nslice) {
    using Acc = typename Traits<P>::Acc;
    constexpr int WTM = BM / WGM, WTN = BM / WGN;
    constexpr int FM = WTM / 16, FN = WTN / 16;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wm = wave / WGN, wn = wave % WGN;
    const int lr = lane & 15, lq = lane >> 4;
    Acc acc[FM][FN];
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int q = 0; q < FN; ++q) acc[f][q] = Acc{};
#pragma unroll 2
    for (int sl = 0; sl < nslice; ++sl) {
        const Acc* src = part + (int64_t)sl * slice_accs<P, BM, WGM, WGN>() + (int64_t)wave * FM * FN * 64;
        Acc v[FM][FN];
#pragma unroll
        for (int f = 0; f < FM; ++f)
#pragma unroll
            for (int q = 0; q < FN; ++q) v[f][q] = src[(f * FN + q) * 64 + lane];
#pragma unroll
        for (int f = 0; f < FM; ++f)
#pragma unroll
            for (int q = 0; q < FN; ++q) acc[f][q] += v[f][q];
    }
    tile_epilogue<P, FM, FN, (RB < FM ? RB : FM)>(g, acc, n, ld, (int64_t)ti * BM + wm * WTM, (int64_t)tj * BM + wn * WTN,
                                                  ti == tj, lr, lq);
}


// Sum of the K pieces of tile (ti, tj) held in slots slot_of(0) .. slot_of(count - 1) of part
// (slots of slice_accs<P, BM, 1, 1>() accumulators; a negative slot is skipped), in that order,
// then the tile's epilogue, by one wavefront.
template <int P, int BM, int RB, class SlotOf>
__device__ __forceinline__ void gemm_tile_fix_slots(const GemmDesc<typename Traits<P>::T>& g, int64_t n, int64_t ld,
                                                    int ti, int tj, const typename Traits<P>::Acc* part, int count,
                                                    SlotOf slot_of) {
    using Acc = typename Traits<P>::Acc;
    constexpr int FM = BM / 16, FN = BM / 16;
    const int lane = threadIdx.x & 63;
    const int lr = lane & 15, lq = lane >> 4;
    Acc acc[FM][FN];
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int q = 0; q < FN; ++q) acc[f][q] = Acc{};
    for (int i = 0; i < count; ++i) {
        const int64_t slot = slot_of(i);
        if (slot < 0) continue;
        const Acc* src = part + slot * slice_accs<P, BM, 1, 1>();
        Acc v[FM][FN];
#pragma unroll
        for (int f = 0; f < FM; ++f)
#pragma unroll
            for (int q = 0; q < FN; ++q) v[f][q] = src[(f * FN + q) * 64 + lane];
#pragma unroll
        for (int f = 0; f < FM; ++f)
#pragma unroll
            for (int q = 0; q < FN; ++q) acc[f][q] += v[f][q];
    }
    tile_epilogue<P, FM, FN, (RB < FM ? RB : FM)>(g, acc, n, ld, (int64_t)ti * BM, (int64_t)tj * BM, ti == tj, lr, lq);
}

}  // namespace
}  // namespace chebdm
