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
// Precisions (KU = k per lane and chunk, loaded as 16-byte vectors):
//   f64     v_mfma_f64_16x16x4f64, KU = 4
//   f32     v_mfma_f32_16x16x4f32, KU = 8
//   bf16x3  v_mfma_f32_16x16x32_bf16 on hi/lo splits of float operands:
//           x = hi + lo, hi = bf16(x), lo = bf16(x - hi); AB ~ hi*hi + hi*lo + lo*hi,
//           float32 accumulation (lo*lo, ~2^-16 relative, is dropped).
//   bf16x6  three-way split x = hi + mid + lo; the six products down to 2^-16
//           relative (hh, hm, mh, hl, lh, mm) keep about float32 accuracy.
#include "gemm_lds.h"
#include "gemm_tile.h"

namespace chebdm {

namespace {

// Work-group -> tile order.  Work-groups are dealt round-robin to the 8 XCDs
// (each with its own L2); with XCD = 1 the linear id is permuted so that each
// XCD walks a contiguous stretch of the row-major upper triangle, whose tiles
// share A row panels in that XCD's L2.
__device__ __forceinline__ int xcd_order(int lin, int total) {
    const int q = total / 8, r = total % 8;
    const int x = lin % 8, slot = lin / 8;
    return x * q + (x < r ? x : r) + slot;
}

template <int XCD>
__device__ __forceinline__ void tile_of_block(int ntri, int& t, int& z) {
    const int gx = gridDim.x;
    int lin = (int)blockIdx.x + (int)blockIdx.z * gx;
    if constexpr (XCD) lin = xcd_order(lin, gx * (int)gridDim.z);
    t = lin % gx;
    z = lin / gx;
    (void)ntri;
}

// Linear tile lin of a grouped launch: product lin / ntri, upper-triangle tile lin % ntri.
__device__ __forceinline__ void lin_tile(int lin, int ntri, int ntile, int& z, int& ti, int& tj) {
    z = lin / ntri;
    upper_tile(lin % ntri, ntile, ti, tj);
}

// BM x BM workgroup tiles, blockIdx.x enumerating the upper triangle, blockIdx.z
// the products of a grouped launch.
// GB > 0: tiles in blocked_tile order with GB x GB super-blocks; 0: row-major.
template <int P, int BM, int WGM, int WGN, int KU, int XCD, int SK = 1, int GB = 0, int RB = 16>
__global__ void __launch_bounds__(64 * WGM * WGN * SK)
k_gemm(const GemmBatch<typename Traits<P>::T> batch, int64_t n, int64_t ld, int64_t kpad, int ntile) {
    int tlin, z;
    tile_of_block<XCD>(ntile * (ntile + 1) / 2, tlin, z);
    int ti, tj;
    if constexpr (GB > 0) blocked_tile(tlin, ntile, GB, ti, tj);
    else upper_tile(tlin, ntile, ti, tj);
    gemm_tile<P, BM, WGM, WGN, KU, SK, RB>(batch.d[z], n, ld, kpad, ti, tj);
}

// Tail split of the register-tile launches (the scheme of the LDS kernel below): full rounds of
// resident work-groups run whole, the few tiles left over run as K slices side by side, and a
// fix-up launch adds the slices in slice order and runs their epilogues.
template <int P, int BM, int WGM, int WGN, int KU, int SK, int RB>
__global__ void __launch_bounds__(64 * WGM * WGN * SK)
k_gemm_main(const GemmBatch<typename Traits<P>::T> batch, int64_t n, int64_t ld, int64_t kpad, int ntile, int ntri) {
    const int lin = xcd_order((int)blockIdx.x, (int)gridDim.x);
    int z, ti, tj;
    lin_tile(lin, ntri, ntile, z, ti, tj);
    gemm_tile<P, BM, WGM, WGN, KU, SK, RB>(batch.d[z], n, ld, kpad, ti, tj);
}

template <int P, int BM, int WGM, int WGN, int KU, int SK, int RB>
__global__ void __launch_bounds__(64 * WGM * WGN * SK)
k_gemm_slice(const GemmBatch<typename Traits<P>::T> batch, int64_t n, int64_t ld, int64_t kpad, int ntile, int ntri,
             int lin0, int nslice, typename Traits<P>::Acc* part) {
    constexpr int CH = 4 * KU;
    const int tile = (int)blockIdx.x / nslice, sl = (int)blockIdx.x % nslice;
    int z, ti, tj;
    lin_tile(lin0 + tile, ntri, ntile, z, ti, tj);
    const int64_t units = kpad / (2 * CH);
    const int64_t k_lo = 2 * CH * (units * sl / nslice), k_hi = 2 * CH * (units * (sl + 1) / nslice);
    gemm_tile<P, BM, WGM, WGN, KU, SK, RB>(batch.d[z], n, ld, kpad, ti, tj, k_lo, k_hi,
                                          part + ((int64_t)tile * nslice + sl) * slice_accs<P, BM, WGM, WGN>());
}

template <int P, int BM, int WGM, int WGN, int RB>
__global__ void __launch_bounds__(64 * WGM * WGN)
k_gemm_fix(const GemmBatch<typename Traits<P>::T> batch, int64_t n, int64_t ld, int ntile, int ntri, int lin0,
           int nslice, const typename Traits<P>::Acc* part) {
    const int tile = (int)blockIdx.x;
    int z, ti, tj;
    lin_tile(lin0 + tile, ntri, ntile, z, ti, tj);
    gemm_tile_fix<P, BM, WGM, WGN, RB>(batch.d[z], n, ld, ti, tj,
                                       part + (int64_t)tile * nslice * slice_accs<P, BM, WGM, WGN>(), nslice);
}

// Stream-K launches of the one-wavefront register tiles.  Of the launch's W tiles, the first dp
// (whole rounds of the G resident work-groups, when what is left still gives every range four K
// units) run whole, tile r + j G on work-group r; the other W - dp tiles times U K units (2 CH
// each) are dealt in equal contiguous ranges to the G work-groups, so the chip runs W / G rounds
// of tile time instead of a whole number of them, and only the tiles of the last partial round
// are cut into pieces.  A tile inside one range runs whole with its epilogue; a tile shared by
// several ranges leaves each piece's raw accumulators in slot 2 r (the first tile of range r) or
// 2 r + 1 (its last), and a fix-up launch adds the pieces in range order (fixed order:
// deterministic) and runs the epilogue.  Ranges go to work-groups in XCD order, so neighbouring
// tiles share an XCD's L2.
__device__ __forceinline__ int64_t sk_range_begin(int64_t total, int64_t r, int64_t G) { return total * r / G; }

template <int P, int BM, int KU, int RB>
__global__ void __launch_bounds__(64)
k_gemm_sk(const GemmBatch<typename Traits<P>::T> batch, int64_t n, int64_t ld, int64_t kpad, int ntile, int ntri,
          int64_t dp, int64_t units, int64_t total, typename Traits<P>::Acc* part) {
    constexpr int CH = 4 * KU;
    const int64_t G = gridDim.x, r = xcd_order((int)blockIdx.x, (int)gridDim.x);
    for (int64_t t = r; t < dp; t += G) {
        int z, ti, tj;
        lin_tile((int)t, ntri, ntile, z, ti, tj);
        gemm_tile<P, BM, 1, 1, KU, 1, RB>(batch.d[z], n, ld, kpad, ti, tj);
    }
    const int64_t a = sk_range_begin(total, r, G), b = sk_range_begin(total, r + 1, G);
    if (a == b) return;
    const int64_t t0 = a / units, t1 = (b - 1) / units;
    for (int64_t t = t0; t <= t1; ++t) {
        const int64_t u0 = (a > t * units ? a : t * units) - t * units;
        const int64_t u1 = (b < (t + 1) * units ? b : (t + 1) * units) - t * units;
        int z, ti, tj;
        lin_tile((int)(dp + t), ntri, ntile, z, ti, tj);
        if (u0 == 0 && u1 == units) {
            gemm_tile<P, BM, 1, 1, KU, 1, RB>(batch.d[z], n, ld, kpad, ti, tj);
        } else {
            const int64_t slot = 2 * r + (t == t0 ? 0 : 1);
            gemm_tile<P, BM, 1, 1, KU, 1, RB>(batch.d[z], n, ld, kpad, ti, tj, u0 * 2 * CH, u1 * 2 * CH,
                                              part + slot * slice_accs<P, BM, 1, 1>());
        }
    }
}

// One work-group per tile past dp; tiles inside one range were finished by k_gemm_sk.
template <int P, int BM, int RB>
__global__ void __launch_bounds__(64)
k_gemm_sk_fix(const GemmBatch<typename Traits<P>::T> batch, int64_t n, int64_t ld, int ntile, int ntri, int64_t dp,
              int64_t units, int64_t total, int64_t G, const typename Traits<P>::Acc* part) {
    const int64_t t = blockIdx.x;
    // range holding iteration i: the largest r with total r / G <= i
    const int64_t ra = ((t * units + 1) * G + total - 1) / total - 1;
    const int64_t rb = (((t + 1) * units) * G + total - 1) / total - 1;
    if (ra == rb) return;
    int z, ti, tj;
    lin_tile((int)(dp + t), ntri, ntile, z, ti, tj);
    gemm_tile_fix_slots<P, BM, RB>(batch.d[z], n, ld, ti, tj, part, (int)(rb - ra + 1), [&](int i) -> int64_t {
        const int64_t r = ra + i;
        const int64_t a = sk_range_begin(total, r, G), b = sk_range_begin(total, r + 1, G);
        if (a == b) return -1;
        return 2 * r + (t == a / units ? 0 : 1);
    });
}

// Stream-K launch over G = 1024 work-groups (one wavefront per SIMD).  sk_fits: the shapes fit,
// the scratch holds 2 G pieces, and every range has at least four K units.
constexpr int64_t kSkGroups = 1024;

template <int P, int BM, int KU>
bool sk_fits(int64_t n, int64_t ld, int count, size_t scratch_bytes) {
    constexpr int CH = 4 * KU;
    const int64_t kpad = (n + 2 * CH - 1) / (2 * CH) * (2 * CH);
    if (kpad > ld || (n + BM - 1) / BM * BM > ld) return false;
    const int64_t ntile = (n + BM - 1) / BM, W = ntile * (ntile + 1) / 2 * count;
    const int64_t need = 2 * kSkGroups * slice_accs<P, BM, 1, 1>() * (int64_t)sizeof(typename Traits<P>::Acc);
    return W * (kpad / (2 * CH)) >= 4 * kSkGroups && need <= (int64_t)scratch_bytes;
}

template <int P, int BM, int KU, int RB = 16>
hipError_t launch_sk(const GemmBatch<typename Traits<P>::T>& b, int64_t n, int64_t ld, hipStream_t st, void* scratch,
                     size_t scratch_bytes) {
    using Acc = typename Traits<P>::Acc;
    constexpr int CH = 4 * KU;
    constexpr int64_t G = kSkGroups;
    if (!scratch || !sk_fits<P, BM, KU>(n, ld, b.count, scratch_bytes)) return hipErrorInvalidValue;
    const int64_t kpad = (n + 2 * CH - 1) / (2 * CH) * (2 * CH);
    const int ntile = (int)((n + BM - 1) / BM);
    const int ntri = ntile * (ntile + 1) / 2;
    const int64_t W = (int64_t)ntri * b.count, units = kpad / (2 * CH);
    int64_t dp = W / G * G;                       // whole rounds run whole ...
    if ((W - dp) * units < 4 * G) dp = 0;         // ... while the rest still gives four units a range
    const int64_t total = (W - dp) * units;
    Acc* part = static_cast<Acc*>(scratch);
    hipLaunchKernelGGL((k_gemm_sk<P, BM, KU, RB>), dim3((unsigned)G), dim3(64), 0, st, b, n, ld, kpad, ntile, ntri,
                       dp, units, total, part);
    hipLaunchKernelGGL((k_gemm_sk_fix<P, BM, RB>), dim3((unsigned)(W - dp)), dim3(64), 0, st, b, n, ld, ntile, ntri,
                       dp, units, total, G, (const Acc*)part);
    return hipGetLastError();
}

// OCC: wavefronts per SIMD the kernel holds (from its register use); the chip's 1024 SIMDs then
// keep 1024 OCC / (WGM WGN SK) work-groups resident.
template <int P, int BM, int WGM, int WGN, int KU, int XCD, int SK = 1, int GB = 0, int RB = 16, int OCC = 1>
hipError_t launch_cfg(const GemmBatch<typename Traits<P>::T>& b, int64_t n, int64_t ld, hipStream_t st,
                      void* scratch = nullptr, size_t scratch_bytes = 0) {
    using Acc = typename Traits<P>::Acc;
    constexpr int CH = 4 * KU;
    const int64_t kpad = (n + 2 * CH - 1) / (2 * CH) * (2 * CH);
    if (kpad > ld || (n + BM - 1) / BM * BM > ld) return hipErrorInvalidValue;
    const int ntile = (int)((n + BM - 1) / BM);
    const int ntri = ntile * (ntile + 1) / 2, total = ntri * b.count;
    const int slots = 1024 * OCC / (WGM * WGN * SK);
    const int rounds = total / slots, rest = total % slots;
    const int64_t units = kpad / (2 * CH);
    int nslice = rest > 0 ? slots / rest : 0;
    if (nslice > 16) nslice = 16;
    if (nslice > units / (8 * SK)) nslice = (int)(units / (8 * SK));
    const int64_t need = (int64_t)rest * nslice * slice_accs<P, BM, WGM, WGN>() * (int64_t)sizeof(Acc);
    const bool split = rounds >= 1 && rest > 0 && rest * 4 <= slots && nslice >= 2 && scratch &&
                       need <= (int64_t)scratch_bytes;
    if (!split) {
        dim3 grid((unsigned)ntri, 1, (unsigned)b.count);
        hipLaunchKernelGGL((k_gemm<P, BM, WGM, WGN, KU, XCD, SK, GB, RB>), grid, dim3(64 * WGM * WGN * SK), 0, st, b,
                           n, ld, kpad, ntile);
        return hipGetLastError();
    }
    Acc* part = static_cast<Acc*>(scratch);
    const int nmain = rounds * slots;
    hipLaunchKernelGGL((k_gemm_main<P, BM, WGM, WGN, KU, SK, RB>), dim3((unsigned)nmain), dim3(64 * WGM * WGN * SK), 0,
                       st, b, n, ld, kpad, ntile, ntri);
    hipLaunchKernelGGL((k_gemm_slice<P, BM, WGM, WGN, KU, SK, RB>), dim3((unsigned)(rest * nslice)),
                       dim3(64 * WGM * WGN * SK), 0, st, b, n, ld, kpad, ntile, ntri, nmain, nslice, part);
    hipLaunchKernelGGL((k_gemm_fix<P, BM, WGM, WGN, RB>), dim3((unsigned)rest), dim3(64 * WGM * WGN), 0, st, b, n, ld,
                       ntile, ntri, nmain, nslice, (const Acc*)part);
    return hipGetLastError();
}

// Split-bf16 products with LDS staging: 128 x 128 tiles, 2 x 2 wavefronts.
template <int P, int XCD, int GB, int DEPTH, int PAD, int SWZ, int LDB, int IGLP>
__global__ void __launch_bounds__(256)
k_gemm_lds(const GemmBatch<float> batch, int64_t n, int64_t ld, int64_t kpad, int ntile) {
    int tlin, z;
    tile_of_block<XCD>(ntile * (ntile + 1) / 2, tlin, z);
    int ti, tj;
    if constexpr (GB > 0) blocked_tile(tlin, ntile, GB, ti, tj);
    else upper_tile(tlin, ntile, ti, tj);
    gemm_tile_lds<P, DEPTH, PAD, SWZ, LDB, IGLP>(batch.d[z], n, ld, kpad, ti, tj);
}

// Tail-split launches.  A grouped launch of W 128-tiles fills the chip in rounds of S
// resident work-groups; when W exceeds a multiple of S by a little, the last round holds a
// few tiles and takes as long as a full one.  Then the first R S tiles (linear order: product
// z = lin / ntri, tile lin % ntri) run whole, and each of the remaining ones is cut into K
// slices run side by side, whose partial accumulators one more launch adds in slice order
// (fixed order: the result does not depend on scheduling) before the tile's epilogue.
template <int P, int DEPTH, int PAD, int SWZ, int LDB, int IGLP>
__global__ void __launch_bounds__(256)
k_gemm_lds_main(const GemmBatch<float> batch, int64_t n, int64_t ld, int64_t kpad, int ntile, int ntri) {
    const int lin = xcd_order((int)blockIdx.x, (int)gridDim.x);
    int z, ti, tj;
    lin_tile(lin, ntri, ntile, z, ti, tj);
    gemm_tile_lds<P, DEPTH, PAD, SWZ, LDB, IGLP>(batch.d[z], n, ld, kpad, ti, tj);
}

constexpr int64_t kSlicePart = 4 * 16 * 64;   // f32x4 per K slice of one tile (64 KB)

template <int P, int DEPTH, int PAD, int SWZ, int LDB, int IGLP>
__global__ void __launch_bounds__(256)
k_gemm_lds_slice(const GemmBatch<float> batch, int64_t n, int64_t ld, int64_t kpad, int ntile, int ntri, int lin0,
                 int nslice, f32x4* part) {
    const int tile = (int)blockIdx.x / nslice, sl = (int)blockIdx.x % nslice;
    int z, ti, tj;
    lin_tile(lin0 + tile, ntri, ntile, z, ti, tj);
    const int64_t units = kpad / 64;   // pairs of 32-wide K steps
    const int64_t s0 = 2 * (units * sl / nslice), s1 = 2 * (units * (sl + 1) / nslice);
    gemm_tile_lds<P, DEPTH, PAD, SWZ, LDB, IGLP>(batch.d[z], n, ld, kpad, ti, tj, s0, s1,
                                                 part + ((int64_t)tile * nslice + sl) * kSlicePart);
}

// one 64-thread work-group per wave tile: four times the work-groups of one per tile
template <int P>
__global__ void __launch_bounds__(64)
k_gemm_lds_fix(const GemmBatch<float> batch, int64_t n, int64_t ld, int ntile, int ntri, int lin0, int nslice,
               const f32x4* part) {
    const int tile = (int)blockIdx.x >> 2, wave = (int)blockIdx.x & 3;
    int z, ti, tj;
    lin_tile(lin0 + tile, ntri, ntile, z, ti, tj);
    gemm_tile_lds_fix<P>(batch.d[z], n, ld, ti, tj, part + (int64_t)tile * nslice * kSlicePart, nslice, wave);
}

// Stream-K launches of the LDS kernel (the scheme of k_gemm_sk): kLdsSlots resident work-groups
// share the launch's tiles x K-step pairs in equal contiguous ranges; pieces of shared tiles
// leave their partials (one tile's kSlicePart per slot) in slot 2 r or 2 r + 1 of range r, and
// k_gemm_lds_sk_fix adds them in range order, one 64-thread work-group per wave tile.
template <int P, int DEPTH, int PAD, int SWZ, int LDB, int IGLP>
__global__ void __launch_bounds__(256)
k_gemm_lds_sk(const GemmBatch<float> batch, int64_t n, int64_t ld, int64_t kpad, int ntile, int ntri, int64_t units,
              int64_t total, f32x4* part) {
    const int64_t G = gridDim.x, r = xcd_order((int)blockIdx.x, (int)gridDim.x);
    const int64_t a = sk_range_begin(total, r, G), b = sk_range_begin(total, r + 1, G);
    if (a == b) return;
    const int64_t t0 = a / units, t1 = (b - 1) / units;
    for (int64_t t = t0; t <= t1; ++t) {
        const int64_t u0 = (a > t * units ? a : t * units) - t * units;
        const int64_t u1 = (b < (t + 1) * units ? b : (t + 1) * units) - t * units;
        int z, ti, tj;
        lin_tile((int)t, ntri, ntile, z, ti, tj);
        if (u0 == 0 && u1 == units) {
            gemm_tile_lds<P, DEPTH, PAD, SWZ, LDB, IGLP>(batch.d[z], n, ld, kpad, ti, tj);
        } else {
            const int64_t slot = 2 * r + (t == t0 ? 0 : 1);
            gemm_tile_lds<P, DEPTH, PAD, SWZ, LDB, IGLP>(batch.d[z], n, ld, kpad, ti, tj, 2 * u0, 2 * u1,
                                                         part + slot * kSlicePart);
        }
        __syncthreads();   // the next tile's panels go into the same LDS stages
    }
}

template <int P>
__global__ void __launch_bounds__(64)
k_gemm_lds_sk_fix(const GemmBatch<float> batch, int64_t n, int64_t ld, int ntile, int ntri, int64_t units,
                  int64_t total, int64_t G, const f32x4* part) {
    const int64_t t = (int64_t)blockIdx.x >> 2;
    const int wave = (int)blockIdx.x & 3;
    const int64_t ra = ((t * units + 1) * G + total - 1) / total - 1;
    const int64_t rb = (((t + 1) * units) * G + total - 1) / total - 1;
    if (ra == rb) return;
    int z, ti, tj;
    lin_tile((int)t, ntri, ntile, z, ti, tj);
    gemm_tile_lds_fix_slots<P>(batch.d[z], n, ld, ti, tj, part, (int)(rb - ra + 1), [&](int i) -> int64_t {
        const int64_t r = ra + i;
        const int64_t a = sk_range_begin(total, r, G), b = sk_range_begin(total, r + 1, G);
        if (a == b) return -1;
        return 2 * r + (t == a / units ? 0 : 1);
    }, wave);
}

// LDS layout: unpadded 64-byte rows with the 16-byte chunks of row r XOR-swizzled by
// (r >> 1) & 3 (measured: 522 -> 570 TFLOP/s of bf16 work at N = 4000 against 8-element padding)
// Rounds of tile work a launch of W tiles takes on S slots: full rounds, plus a small tail when
// the last round is split into K slices (under a quarter full, after a full round), else one more.
__host__ inline double rounds_of(int64_t W, int64_t S) {
    const int64_t full = W / S, rest = W % S;
    if (rest == 0) return (double)full;
    return (double)full + ((full >= 1 && rest * 4 <= S) ? 0.15 : 1.0);
}

// 64-tiles from one full round on: one wavefront per tile (1024 slots) or the K split over two
// (512 slots, half a tile's time each, plus the split's cost `over`), whichever quantises better
// (N = 1500 eight products, float64: 44.2 -> 50.0 TFLOP/s; N = 3000 four: 54.0 -> 58.9).
__host__ inline bool k_split_quantises_better(int64_t w64, double over) {
    return rounds_of(w64, 512) * 0.5 * over < rounds_of(w64, 1024);
}

// Resident work-groups of the LDS kernel: two per CU (two wavefronts per SIMD, <= 80 KB of LDS).
constexpr int kLdsSlots = 2 * 256;

template <int P, int XCD, int GB, int DEPTH = 2, int PAD = 0, int SWZ = 1, int LDB = 1, int IGLP = -1>
hipError_t launch_lds(const GemmBatch<float>& b, int64_t n, int64_t ld, hipStream_t st, f32x4* scratch = nullptr,
                      int64_t scratch_vec = 0) {
    const int64_t kpad = (n + 63) / 64 * 64;
    const int ntile = (int)((n + 127) / 128);
    if (kpad > ld || (int64_t)ntile * 128 > ld) return hipErrorInvalidValue;
    const int ntri = ntile * (ntile + 1) / 2;
    const int total = ntri * b.count;
    const int rounds = total / kLdsSlots, rest = total % kLdsSlots;
    // tail split: a last round under a quarter full, at least 8 K-step pairs per slice
    int nslice = rest > 0 ? kLdsSlots / rest : 0;
    if (nslice > 16) nslice = 16;
    if (nslice > kpad / 64 / 8) nslice = (int)(kpad / 64 / 8);
    const bool split = rounds >= 1 && rest > 0 && rest * 4 <= kLdsSlots && nslice >= 2 && scratch &&
                       (int64_t)rest * nslice * kSlicePart <= scratch_vec;
    if (!split) {
        dim3 grid((unsigned)ntri, 1, (unsigned)b.count);
        hipLaunchKernelGGL((k_gemm_lds<P, XCD, GB, DEPTH, PAD, SWZ, LDB, IGLP>), grid, dim3(256), 0, st, b, n, ld,
                           kpad, ntile);
        return hipGetLastError();
    }
    const int nmain = rounds * kLdsSlots;
    hipLaunchKernelGGL((k_gemm_lds_main<P, DEPTH, PAD, SWZ, LDB, IGLP>), dim3((unsigned)nmain), dim3(256), 0, st, b, n,
                       ld, kpad, ntile, ntri);
    hipLaunchKernelGGL((k_gemm_lds_slice<P, DEPTH, PAD, SWZ, LDB, IGLP>), dim3((unsigned)(rest * nslice)), dim3(256),
                       0, st, b, n, ld, kpad, ntile, ntri, nmain, nslice, scratch);
    hipLaunchKernelGGL((k_gemm_lds_fix<P>), dim3((unsigned)(rest * 4)), dim3(64), 0, st, b, n, ld, ntile, ntri, nmain,
                       nslice, (const f32x4*)scratch);
    return hipGetLastError();
}

// Stream-K over kLdsSlots work-groups: the shapes fit, the scratch holds 2 kLdsSlots tile
// partials, and every range has at least four K-step pairs.
inline bool lds_sk_fits(int64_t n, int64_t ld, int count, int64_t scratch_vec) {
    const int64_t kpad = (n + 63) / 64 * 64, ntile = (n + 127) / 128;
    if (kpad > ld || ntile * 128 > ld) return false;
    const int64_t W = ntile * (ntile + 1) / 2 * count;
    return W * (kpad / 64) >= 4 * (int64_t)kLdsSlots && 2 * (int64_t)kLdsSlots * kSlicePart <= scratch_vec;
}

template <int P, int DEPTH, int PAD, int SWZ, int LDB, int IGLP>
hipError_t launch_lds_sk(const GemmBatch<float>& b, int64_t n, int64_t ld, hipStream_t st, f32x4* scratch,
                         int64_t scratch_vec) {
    if (!scratch || !lds_sk_fits(n, ld, b.count, scratch_vec)) return hipErrorInvalidValue;
    const int64_t kpad = (n + 63) / 64 * 64;
    const int ntile = (int)((n + 127) / 128), ntri = ntile * (ntile + 1) / 2;
    const int64_t W = (int64_t)ntri * b.count, units = kpad / 64, total = W * units, G = kLdsSlots;
    hipLaunchKernelGGL((k_gemm_lds_sk<P, DEPTH, PAD, SWZ, LDB, IGLP>), dim3((unsigned)G), dim3(256), 0, st, b, n, ld,
                       kpad, ntile, ntri, units, total, scratch);
    hipLaunchKernelGGL((k_gemm_lds_sk_fix<P>), dim3((unsigned)(W * 4)), dim3(64), 0, st, b, n, ld, ntile, ntri, units,
                       total, G, (const f32x4*)scratch);
    return hipGetLastError();
}

// Launch configuration, from a measured sweep on MI355X (N = 1000 / 2000 / 4000, one and
// four products per launch).  One wavefront per tile in every choice (64-thread work-groups
// per K slice), XCD-ordered.  What decides is how well the launch fills the 1024 SIMDs:
// these kernels hold one wavefront per SIMD (their accumulators and two register stages
// take more than half of the 512 registers), so a launch of W wavefronts runs in
// ceil(W / 1024) waves of work.  With few 64-tiles (W64 = upper-triangle 64-tiles x
// products) smaller 48-tiles and K split over 2 or 4 wavefronts (summed through LDS) fill the
// chip better; with many, 64-tiles without a split are fastest.  Measured (algorithmic
// TFLOP/s, float64): N = 1000 single product 16 -> 31 (48-tiles, K split 4); N = 1000 four
// products 28 -> 42 (48-tiles); N = 2000 single 28 -> 45 (48-tiles); N = 4000: 64-tiles.
// 48-tiles need ceil(n/48)*48 <= ld; otherwise 64-tiles are used.
template <int P>
hipError_t launch_any(const GemmBatch<typename Traits<P>::T>& b, int64_t n, int64_t ld, hipStream_t st,
                      void* scratch = nullptr, size_t scratch_bytes = 0) {
    if (b.count <= 0) return hipSuccess;
    if (b.count > kMaxGroup || ld % 128 != 0) return hipErrorInvalidValue;
    constexpr int KU = P == P_F64 ? 4 : (P == P_F32 ? 8 : 16);
    const int64_t t64 = (n + 63) / 64;
    const int64_t w64 = t64 * (t64 + 1) / 2 * b.count;
    const bool fits48 = (n + 47) / 48 * 48 <= ld;
    const int64_t t48 = (n + 47) / 48, w48 = t48 * (t48 + 1) / 2 * b.count;
    // With at least one full round of 64-tiles (w64 >= 1024) the unsplit 64-tile kernel with the
    // tail split wins (N = 2000, TFLOP/s, two / four / eight products: float64 48.8 / 53.1 / 55.7
    // against 46.3 / 46.6 / 51.7 for 48-tiles; float32 82.6 / 96.7 / 106.7 against 61.6 / 58.0 /
    // 60.9); below it the smaller 48-tiles fill the chip better (float64 N = 2000 single: 40.0
    // against 38.4 for split 64-tiles; N = 1000: 48-tiles, K split 4 ways up to 300 64-tiles).
    // Stream-K from N = 1500 (K long enough for pieces) while the 64-tiles fill less than three
    // rounds and leave the last one under 80 % full: one product at N = 1500 / 2000, float64
    // 0.094 / 0.186 ms against 0.126 / 0.196, float32 0.067 / 0.111 against 0.088 / 0.135;
    // three products at N = 2000, float32 0.257 against 0.294; no gain from three full rounds
    // on (N = 2000, eight products) or with a nearly full last round (N = 4000, one product).
    // Float32 also from N = 1000 once the 64-tiles fill one round (eight products at N = 1000:
    // 0.129 -> 0.105 ms).  Past one round, a last round under a quarter full goes to the tail
    // split instead, for float64 from N = 1500 (N = 2000, two / four products: 0.345 / 0.631 ->
    // 0.333 / 0.596 ms; N = 3000, one / two: 0.556 / 0.995 -> 0.510 / 0.929) and for float32 from
    // N = 2500 (N = 3000, one / two: 0.296 / 0.536 -> 0.278 / 0.504; at N = 2000, two products,
    // stream-K stays ahead, 0.184 against 0.195, and at N = 1000 the K slices are too short).
    if constexpr (P == P_F64 || P == P_F32) {
        const bool long_enough = n >= 1500 || (P == P_F32 && w64 >= 1024);
        const bool tail_split_fits =
            n >= (P == P_F64 ? 1500 : 2500) && w64 >= 1024 && (w64 % 1024) * 4 <= 1024;
        if (long_enough && !tail_split_fits && scratch && w64 < 3 * 1024 && w64 % 1024 < 820 &&
            sk_fits<P, 64, KU>(n, ld, b.count, scratch_bytes))
            return launch_sk<P, 64, KU>(b, n, ld, st, scratch, scratch_bytes);
    }
    if constexpr (P == P_F64) {
        if (w64 >= 1024 && n >= 1500) {
            if (k_split_quantises_better(w64, 1.10))
                return launch_cfg<P, 64, 1, 1, KU, 1, 2>(b, n, ld, st, scratch, scratch_bytes);
            return launch_cfg<P, 64, 1, 1, KU, 1, 1>(b, n, ld, st, scratch, scratch_bytes);
        }
        // 48-tiles while about one round of them (one wavefront per SIMD) holds the launch; past
        // that, up to one round of 64-tiles beats two rounds of 48-tiles (N = 1000, six / seven
        // products: 0.147 against 0.183 / 0.185 ms; N = 1500, three: 0.211 against 0.264)
        if (fits48 && w48 <= 1200) {
            if (w64 < 300) return launch_cfg<P, 48, 1, 1, KU, 1, 4>(b, n, ld, st, scratch, scratch_bytes);
            return launch_cfg<P, 48, 1, 1, KU, 1, 1>(b, n, ld, st, scratch, scratch_bytes);
        }
        if (!fits48 && w64 < 400) return launch_cfg<P, 64, 1, 1, KU, 1, 4>(b, n, ld, st, scratch, scratch_bytes);
        if (w64 <= 1024) {
            if (k_split_quantises_better(w64, 1.10))
                return launch_cfg<P, 64, 1, 1, KU, 1, 2>(b, n, ld, st, scratch, scratch_bytes);
            return launch_cfg<P, 64, 1, 1, KU, 1, 1>(b, n, ld, st, scratch, scratch_bytes);
        }
        if (fits48) return launch_cfg<P, 48, 1, 1, KU, 1, 1>(b, n, ld, st, scratch, scratch_bytes);
        return launch_cfg<P, 64, 1, 1, KU, 1, 1>(b, n, ld, st, scratch, scratch_bytes);
    } else if constexpr (P == P_F32) {
        if (w64 >= 1024) {
            if (k_split_quantises_better(w64, 1.15))
                return launch_cfg<P, 64, 1, 1, KU, 1, 2>(b, n, ld, st, scratch, scratch_bytes);
            return launch_cfg<P, 64, 1, 1, KU, 1, 1>(b, n, ld, st, scratch, scratch_bytes);
        }
        // 48-tiles split over two wavefronts while one round of them holds the launch; past that
        // 64-tiles (N = 1000, five / six / seven products: 0.077 / 0.082 / 0.084 against 0.093 /
        // 0.108 / 0.132 ms; N = 1500, two / three: 0.110 / 0.118 against 0.132 / 0.186), split
        // over two wavefronts only while that still fits one round
        // With the accumulators in VGPRs the float32 48-tile holds two wavefronts per SIMD, and
        // past the smallest launches it runs best unsplit (N = 1000, two / three / four products:
        // 0.049 / 0.069 / 0.085 -> 0.044 / 0.047 / 0.056 ms; one product stays split: 0.027
        // against 0.042)
        if (fits48 && w48 <= 300) return launch_cfg<P, 48, 1, 1, KU, 1, 2, 0, 16, 2>(b, n, ld, st, scratch, scratch_bytes);
        if (fits48 && w48 <= 1024) return launch_cfg<P, 48, 1, 1, KU, 1, 1, 0, 16, 2>(b, n, ld, st, scratch, scratch_bytes);
        if (w64 < 512) return launch_cfg<P, 64, 1, 1, KU, 1, 2>(b, n, ld, st, scratch, scratch_bytes);
        return launch_cfg<P, 64, 1, 1, KU, 1, 1>(b, n, ld, st, scratch, scratch_bytes);
    } else {
        // LDS staging (each element split once per work-group, panels two K steps ahead) once
        // there are >= 100 128-tiles: three-term split at N = 4000 390 -> 563 TFLOP/s of bf16
        // work, N = 2000 four products 289 -> 532.  Three-term: two LDS stages (one barrier per
        // K step) and the compiler's MFMA/LDS interleave (iglp 0), 591 -> 617 at N = 4000;
        // six-term: interleave only (two stages would take 96 KB of LDS, one work-group per
        // CU), 742 -> 754.  With the tail split the six-term LDS kernel also wins for single
        // products (mu search + D, N = 4000: 27.2 -> 36.1 DM/s; N = 2000: 105.9 -> 119.7).
        const int64_t t128 = (n + 127) / 128, w128 = t128 * (t128 + 1) / 2 * b.count;
        f32x4* sc = static_cast<f32x4*>(scratch);
        const int64_t sv = (int64_t)(scratch_bytes / sizeof(f32x4));
        // stream-K on the LDS kernel from N = 1500 while the 128-tiles fill under 80 % of one round
        // of kLdsSlots (mu search + D at N = 2000: three-term 194 -> 223 DM/s, six-term 130 ->
        // 150); past one round the tail split is better (N = 4000, one product of 528 tiles,
        // as stream-K: mu search + D 54 -> 41 DM/s)
        const bool lds_sk = n >= 1500 && w128 < 410 && sc && lds_sk_fits(n, ld, b.count, sv);
        if constexpr (P == P_BF16X3) {
            if (w128 >= 100 && lds_sk) return launch_lds_sk<P, 2, 0, 1, 2, 0>(b, n, ld, st, sc, sv);
            if (w128 >= 100) return launch_lds<P, 1, 0, 2, 0, 1, 2, 0>(b, n, ld, st, sc, sv);
        } else {
            if (w128 >= 120 && lds_sk) return launch_lds_sk<P, 2, 0, 1, 1, 0>(b, n, ld, st, sc, sv);
            // (N = 1000, three products, 108 128-tiles: 0.068 ms against 0.058 for split 64-tiles)
            if (w128 >= 120) return launch_lds<P, 1, 0, 2, 0, 1, 1, 0>(b, n, ld, st, sc, sv);
        }
        // the smallest launches on 48-tiles split over two wavefronts (N = 1000, one / two
        // products: three-term 0.022 / 0.034 ms, six-term 0.029 / 0.041, against 0.035 / 0.048 and
        // 0.045 / 0.057 for split 64-tiles; N = 1500, one product of 528 48-tiles: 0.067 and 0.082
        // against 0.063 and 0.074)
        if (fits48 && w48 <= 500)
            return launch_cfg<P, 48, 1, 1, KU, 1, 2, 0, 16, 2>(b, n, ld, st, scratch, scratch_bytes);
        // below a full round of 64-tiles the K split over two wavefronts fills the chip better
        // (N = 1500, mu search + D: six-term 148 -> 192 DM/s, three-term 217 -> 223)
        if (w64 < 1024) return launch_cfg<P, 64, 1, 1, KU, 1, 2>(b, n, ld, st, scratch, scratch_bytes);
        return launch_cfg<P, 64, 1, 1, KU, 1, 1>(b, n, ld, st, scratch, scratch_bytes);
    }
}

}  // namespace

hipError_t launch_gemm_f64(const GemmBatch<double>& b, int64_t n, int64_t ld, hipStream_t st, void* scratch,
                           size_t scratch_bytes) {
    return launch_any<P_F64>(b, n, ld, st, scratch, scratch_bytes);
}

hipError_t launch_gemm_f32(const GemmBatch<float>& b, int64_t n, int64_t ld, int split, hipStream_t st,
                           void* scratch, size_t scratch_bytes) {
    if (split == 2) return launch_any<P_BF16X6>(b, n, ld, st, scratch, scratch_bytes);
    if (split == 1) return launch_any<P_BF16X3>(b, n, ld, st, scratch, scratch_bytes);
    return launch_any<P_F32>(b, n, ld, st, scratch, scratch_bytes);
}

}  // namespace chebdm
