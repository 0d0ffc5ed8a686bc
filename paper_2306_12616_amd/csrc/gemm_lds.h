// LDS-staged tile routine for the split-bf16 precisions.
//
// The register-direct routine (gemm_tile) splits every float32 operand into
// bf16 terms inside each wavefront, once per use, and streams its operands
// from L2 per wavefront; for the split precisions that makes the VALU split
// work and the operand traffic, not the MFMA units, the bound.  Here a
// work-group of 2 x 2 wavefronts owns a 128 x 128 tile: per K step of 32 it
// loads the 128-row A and B panels once (float32, 16-byte loads), splits each
// element once into its bf16 terms, stores the terms in LDS, and every
// wavefront reads its 64 x 64 operands from LDS (each panel row is used by two
// wavefronts).  Same K order in both operands, same float32 accumulation and
// the same fused epilogue as gemm_tile.
#pragma once

#include "gemm_tile.h"

namespace chebdm {
namespace {

template <int P>
struct SplitTerms;
template <>
struct SplitTerms<P_BF16X3> {
    static constexpr int N = 2;
};
template <>
struct SplitTerms<P_BF16X6> {
    static constexpr int N = 3;
};

// One 128 x 128 tile (ti, tj), ti <= tj, by the calling 256-thread work-group.
// kpad: K padded to a multiple of 2*32 = 64, kpad <= ld; rows ti*128 .. +127 and
// tj*128 .. +127 must lie inside the ld x ld operands.
// DEPTH = 1: the panels of step s+1 are loaded while step s computes; DEPTH = 2:
// those of step s+2 (two register stages, the loop body unrolled by two).
// LDS rows are KC + PAD bf16 long; SWZ > 0 XORs the 16-byte chunk index of row r with
// (r >> SWZ) & 3 (a bank swizzle; use with PAD = 0).
// LDB = 2 keeps two LDS stages: step s + 1 is written into one while step s is read from the
// other, so one barrier per K step suffices (LDB = 1: two, around the single stage).  With
// DEPTH = 2 the last two steps run after the loop, without the clamped loads, LDS stores and
// barriers a further trip would spend on steps past the end (split products at N = 2000 /
// 4000: 2 % / 1 % faster).
template <int P, int DEPTH = 2, int PAD = 8, int SWZ = 0, int LDB = 1, int IGLP = -1>
__device__ __forceinline__ void gemm_tile_lds(const GemmDesc<float>& g, int64_t n, int64_t ld, int64_t kpad, int ti,
                                              int tj, int64_t s0 = 0, int64_t s1 = -1, f32x4* part = nullptr) {
    static_assert(P == P_BF16X3 || P == P_BF16X6, "split-bf16 precisions only");
    static_assert(DEPTH == 1 || DEPTH == 2, "prefetch depth 1 or 2");
    static_assert(LDB == 1 || (LDB == 2 && DEPTH == 2), "two LDS stages need two register stages");
    using Acc = f32x4;
    constexpr int BM = 128, KC = 32, NT = SplitTerms<P>::N, RS = KC + PAD;
    __shared__ __attribute__((aligned(16))) __bf16 lds[LDB][2][NT][BM][RS];
    // column (in bf16) of 16-byte chunk c of row r
    auto col = [](int r, int c) -> int { return SWZ > 0 ? 8 * (c ^ ((r >> SWZ) & 3)) : 8 * c; };

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int lr = lane & 15, lq = lane >> 4;
    const bool diag_tile = ti == tj;
    const bool idle = diag_tile && wm > wn;   // this wave's 64 x 64 lies below the diagonal

    // staging: thread -> row tid/2 of both panels, 16 consecutive k at (tid%2)*16
    const int srow = tid >> 1, sk = (tid & 1) * 16;
    const float* __restrict__ ga = g.A + ((int64_t)ti * BM + srow) * ld + sk;
    const float* __restrict__ gb = g.B + ((int64_t)tj * BM + srow) * ld + sk;
    // K steps [s0, s1) of KC (s1 < 0: all); both even
    const int64_t steps = s1 < 0 ? kpad / KC : s1;
    struct Stage {
        f32x4 a[4], b[4];
    };
    auto gload = [&](Stage& r, int64_t s) {
        const int64_t k0 = (s < steps ? s : steps - 1) * KC;   // clamped: no branch in the loop
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            r.a[c] = *reinterpret_cast<const f32x4*>(ga + k0 + 4 * c);
            r.b[c] = *reinterpret_cast<const f32x4*>(gb + k0 + 4 * c);
        }
    };
    auto put1 = [&](int buf, int which, const f32x4 (&r)[4]) {
        float x[16];
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int t = 0; t < 4; ++t) x[4 * c + t] = r[c][t];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            bf16x8 t0, t1, t2;
            if constexpr (NT == 2) split_bf16(&x[8 * h], t0, t1);
            else split3_bf16(&x[8 * h], t0, t1, t2);
            const int cc = col(srow, sk / 8 + h);
            *reinterpret_cast<bf16x8*>(&lds[buf][which][0][srow][cc]) = t0;
            *reinterpret_cast<bf16x8*>(&lds[buf][which][1][srow][cc]) = t1;
            if constexpr (NT == 3) *reinterpret_cast<bf16x8*>(&lds[buf][which][2][srow][cc]) = t2;
        }
    };
    auto put = [&](const Stage& r, int buf = 0) {
        put1(buf, 0, r.a);
        put1(buf, 1, r.b);
    };

    Acc acc[4][4];
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[f][q] = Acc{};

    auto compute = [&](int buf = 0) {
        if (idle) return;
        if constexpr (IGLP >= 0) __builtin_amdgcn_iglp_opt(IGLP);
        bf16x8 a[NT][4], b[NT][4];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const int ra = wm * 64 + f * 16 + lr, rb = wn * 64 + f * 16 + lr;
                a[t][f] = *reinterpret_cast<const bf16x8*>(&lds[buf][0][t][ra][col(ra, lq)]);
                b[t][f] = *reinterpret_cast<const bf16x8*>(&lds[buf][1][t][rb][col(rb, lq)]);
            }
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if constexpr (NT == 2) {
                    acc[f][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][f], b[0][q], acc[f][q], 0, 0, 0);
                    acc[f][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][f], b[1][q], acc[f][q], 0, 0, 0);
                    acc[f][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][f], b[0][q], acc[f][q], 0, 0, 0);
                } else {
                    acc[f][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2][f], b[0][q], acc[f][q], 0, 0, 0);
                    acc[f][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][f], b[2][q], acc[f][q], 0, 0, 0);
                    acc[f][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][f], b[1][q], acc[f][q], 0, 0, 0);
                    acc[f][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][f], b[0][q], acc[f][q], 0, 0, 0);
                    acc[f][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][f], b[1][q], acc[f][q], 0, 0, 0);
                    acc[f][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][f], b[0][q], acc[f][q], 0, 0, 0);
                }
            }
    };

    if constexpr (DEPTH == 1) {
        Stage r;
        gload(r, s0);
        put(r);
        __syncthreads();
        for (int64_t s = s0; s < steps; ++s) {
            gload(r, s + 1);
            compute();
            __syncthreads();
            put(r);
            __syncthreads();
        }
    } else if constexpr (LDB == 2) {
        // steps is even; stage 0 holds even steps, stage 1 odd ones
        Stage r0, r1;
        gload(r0, s0);
        gload(r1, s0 + 1);
        put(r0, 0);
        gload(r0, s0 + 2);
        __syncthreads();
        for (int64_t s = s0; s + 2 < steps; s += 2) {
            compute(0);         // step s
            put(r1, 1);         // step s + 1: stage 1 was last read before the previous barrier
            gload(r1, s + 3);
            __syncthreads();
            compute(1);         // step s + 1
            put(r0, 0);         // step s + 2
            gload(r0, s + 4);
            __syncthreads();
        }
        compute(0);             // the last two steps
        put(r1, 1);
        __syncthreads();
        compute(1);
    } else {
        // steps is even (kpad is a multiple of 64)
        Stage r0, r1;
        gload(r0, s0);
        gload(r1, s0 + 1);
        put(r0);
        __syncthreads();
        for (int64_t s = s0; s + 2 < steps; s += 2) {
            gload(r0, s + 2);   // r0 was consumed: fetch two steps ahead
            compute();          // step s
            __syncthreads();
            put(r1);            // step s + 1
            __syncthreads();
            gload(r1, s + 3);
            compute();          // step s + 1
            __syncthreads();
            put(r0);            // step s + 2
            __syncthreads();
        }
        compute();              // the last two steps
        __syncthreads();
        put(r1);
        __syncthreads();
        compute();
    }
    if (part) {
        // a K slice of the tile: the raw accumulators, lane-native, wave by wave
        if (!idle) {
            f32x4* dst = part + (int64_t)wave * 16 * 64;
#pragma unroll
            for (int f = 0; f < 4; ++f)
#pragma unroll
                for (int q = 0; q < 4; ++q) dst[(f * 4 + q) * 64 + lane] = acc[f][q];
        }
        return;
    }
    // one block row at a time: keeps the kernel within two wavefronts per SIMD, which
    // lets two work-groups per CU alternate around their barriers
    if (!idle)
        tile_epilogue<P, 4, 4, 1>(g, acc, n, ld, (int64_t)ti * BM + wm * 64, (int64_t)tj * BM + wn * 64, diag_tile,
                                  lr, lq);
}

// Sum of the K-slice partials of one 64 x 64 wave tile (wave 0..3 of the 2 x 2 layout of
// gemm_tile_lds) in slice order, then its epilogue, by the calling wavefront.
template <int P>
__device__ __forceinline__ void gemm_tile_lds_fix(const GemmDesc<float>& g, int64_t n, int64_t ld, int ti, int tj,
                                                  const f32x4* part, int nslice, int wave) {
    constexpr int BM = 128;
    const int lane = threadIdx.x & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int lr = lane & 15, lq = lane >> 4;
    const bool diag_tile = ti == tj;
    if (diag_tile && wm > wn) return;
    f32x4 acc[4][4];
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[f][q] = f32x4{};
#pragma unroll 4
    for (int sl = 0; sl < nslice; ++sl) {
        const f32x4* src = part + ((int64_t)sl * 4 + wave) * 16 * 64;
        f32x4 v[4][4];
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int q = 0; q < 4; ++q) v[f][q] = src[(f * 4 + q) * 64 + lane];
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[f][q] += v[f][q];
    }
    tile_epilogue<P, 4, 4, 1>(g, acc, n, ld, (int64_t)ti * BM + wm * 64, (int64_t)tj * BM + wn * 64, diag_tile, lr,
                              lq);
}

// As gemm_tile_lds_fix, with the K pieces of the tile in slots slot_of(0) .. slot_of(count - 1)
// of part (one 128 x 128 tile's partials, kSlicePart-sized, per slot; a negative slot is
// skipped), added in that order.
template <int P, class SlotOf>
__device__ __forceinline__ void gemm_tile_lds_fix_slots(const GemmDesc<float>& g, int64_t n, int64_t ld, int ti,
                                                        int tj, const f32x4* part, int count, SlotOf slot_of,
                                                        int wave) {
    constexpr int BM = 128;
    const int lane = threadIdx.x & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int lr = lane & 15, lq = lane >> 4;
    const bool diag_tile = ti == tj;
    if (diag_tile && wm > wn) return;
    f32x4 acc[4][4];
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[f][q] = f32x4{};
    for (int i = 0; i < count; ++i) {
        const int64_t slot = slot_of(i);
        if (slot < 0) continue;
        const f32x4* src = part + (slot * 4 + wave) * 16 * 64;
        f32x4 v[4][4];
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int q = 0; q < 4; ++q) v[f][q] = src[(f * 4 + q) * 64 + lane];
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[f][q] += v[f][q];
    }
    tile_epilogue<P, 4, 4, 1>(g, acc, n, ld, (int64_t)ti * BM + wm * 64, (int64_t)tj * BM + wn * 64, diag_tile, lr,
                              lq);
}

}  // namespace
}  // namespace chebdm
