// Batched path: many Hamiltonians of different n in one sequence of launches
// (captured once into a HIP graph by the host).  Every kernel takes the
// per-problem geometry table (sizes, workspace offsets, tile choice) and the
// run-time problem table (the caller's H and D pointers, beta, N_e); grids
// span the largest problem and threads outside a problem's n exit.
//
// The matrix products use a persistent kernel per product step: a resident
// grid of one-wavefront work-groups claims (problem, tile) items from an
// atomic counter in the order the tuner chose, and runs the same tile
// routine as the single-problem kernel (with each problem's tile edge).
// Dependencies between steps are kernel boundaries; inside a step the items
// are independent.  (Finer-grained dependencies inside one kernel would need
// agent-scope acquire/release between work-groups, which on the multi-XCD
// gfx950 writes back and invalidates L2 at every wait.)
#include "cheb_dev.h"
#include "gemm_tile.h"
#include "reduce.h"
#include "search_dev.h"

namespace chebdm {

namespace {

typedef double f64x2b __attribute__((ext_vector_type(2)));

template <int P> struct BatchKU;   // k per lane per chunk for the 64-, 48- and 32-edge tiles
template <> struct BatchKU<P_F64> { static constexpr int K64 = 4, K32 = 4; };
template <> struct BatchKU<P_F32> { static constexpr int K64 = 8, K32 = 8; };
template <> struct BatchKU<P_BF16X3> { static constexpr int K64 = 16, K32 = 16; };
template <> struct BatchKU<P_BF16X6> { static constexpr int K64 = 16, K32 = 16; };

template <int P>
__global__ void __launch_bounds__(64)
k_batch_gemm(const GemmDesc<typename Traits<P>::T>* __restrict__ descs, const BatchGeom* __restrict__ geo,
             const TileItem* __restrict__ items, int nitems, int* __restrict__ counter) {
    constexpr int KU64 = BatchKU<P>::K64, KU32 = BatchKU<P>::K32;
    // diagonal wave tiles skip their below-diagonal blocks (the claimed items even the load out);
    // the split-bf16 loops would spill registers with the second loop copy, so they keep one
    constexpr bool kDS = P == P_F64 || P == P_F32;
    for (;;) {
        int idx = 0;
        if (threadIdx.x == 0) idx = atomicAdd(counter, 1);
        idx = __shfl(idx, 0, 64);
        if (idx >= nitems) break;
        const TileItem it = items[idx];
        const BatchGeom gm = geo[it.p];
        const GemmDesc<typename Traits<P>::T> g = descs[it.p];
        int ti, tj;
        upper_tile(it.t, gm.ntile, ti, tj);
        // A tile of the last tile column whose columns end within its first half runs as the left
        // wave tile of a 1 x 2 split (the right half is all padding); a single wavefront may do
        // that because an unsplit K range has no barrier.
        const bool half = tj == gm.ntile - 1 && gm.n - (int64_t)tj * gm.tile <= gm.tile / 2;
        if (gm.tile == 64) {
            const int64_t kpad = (gm.n + 8 * KU64 - 1) / (8 * KU64) * (8 * KU64);
            if (half) gemm_tile<P, 64, 1, 2, KU64>(g, gm.n, gm.ld, kpad, ti, tj);
            else gemm_tile<P, 64, 1, 1, KU64, 1, 16, -1, kDS>(g, gm.n, gm.ld, kpad, ti, tj);
        } else if (gm.tile == 48) {   // only where ceil(n / 48) * 48 <= ld (the host checks)
            const int64_t kpad = (gm.n + 8 * KU64 - 1) / (8 * KU64) * (8 * KU64);
            gemm_tile<P, 48, 1, 1, KU64, 1, 16, -1, kDS>(g, gm.n, gm.ld, kpad, ti, tj);
        } else {
            const int64_t kpad = (gm.n + 8 * KU32 - 1) / (8 * KU32) * (8 * KU32);
            if (half) gemm_tile<P, 32, 1, 2, KU32>(g, gm.n, gm.ld, kpad, ti, tj);
            else gemm_tile<P, 32, 1, 1, KU32, 1, 16, -1, kDS>(g, gm.n, gm.ld, kpad, ti, tj);
        }
    }
}

__global__ void k_batch_zero(int* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// ---- bounds: column sums of |H| (symmetric: equal to row sums), then min/max per problem
__global__ void __launch_bounds__(256)
k_batch_colsum(const BatchProblem* __restrict__ tab, const BatchGeom* __restrict__ geo, double* __restrict__ colsum) {
    const int p = blockIdx.y;
    const int64_t n = geo[p].n;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const double* __restrict__ H = tab[p].H;
    const int64_t ldh = tab[p].ldh;
    double s = 0.0;
#pragma unroll 8
    for (int64_t i = 0; i < n; ++i) {
        const double v = fabs(H[i * ldh + j]);
        s += (i == j) ? 0.0 : v;
    }
    colsum[geo[p].col_off + j] = s;
}

__global__ void __launch_bounds__(256)
k_batch_bounds_final(const BatchProblem* __restrict__ tab, const BatchGeom* __restrict__ geo,
                     const double* __restrict__ colsum, DevScalars* s) {
    __shared__ double smem[4];
    const int p = blockIdx.x;
    const int64_t n = geo[p].n;
    const double* __restrict__ H = tab[p].H;
    const int64_t ldh = tab[p].ldh;
    double lo = INFINITY, hi = -INFINITY;
    int bad = 0;
    for (int64_t j = threadIdx.x; j < n; j += 256) {
        const double r = colsum[geo[p].col_off + j], d = H[j * ldh + j];
        if (!isfinite(r) || !isfinite(d)) bad = 1;
        lo = fmin(lo, d - r);
        hi = fmax(hi, d + r);
    }
    const double nb = block_sum<256>((double)bad, smem);
    lo = block_min<256>(lo, smem);
    hi = block_max<256>(hi, smem);
    if (threadIdx.x == 0) {
        s[p].emin = lo;
        s[p].emax = hi;
        s[p].nonfinite = nb > 0.0 ? 1 : 0;
    }
}

// Per-problem scaling, quadrature size and validity.  status: 0 ok, 2 scalar H (e_a = e_b),
// CHEBDM_ERR_NONFINITE, CHEBDM_ERR_ARG (N_e outside (0, n) or M above the plan's cap).
__global__ void k_batch_setup(const BatchProblem* __restrict__ tab, const BatchGeom* __restrict__ geo,
                              DevScalars* s, int64_t* mq, int count, int order, int64_t mcap, double tol,
                              int max_iter) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= count) return;
    DevScalars& d = s[p];
    const double cen = 0.5 * (d.emin + d.emax), half = 0.5 * (d.emax - d.emin);
    d.cen = cen;
    d.half = half;
    d.beta_s = tab[p].beta * half;
    d.mu_s = 0.0;
    d.n_elec = tab[p].n_elec;
    d.tol = tol;
    d.max_iter = max_iter;
    d.iters = 0;
    d.trace = 0.0;
    int st = 0;
    int64_t M = quad_rule(order, d.beta_s);
    if (d.nonfinite) st = CHEBDM_ERR_NONFINITE;
    else if (!(tab[p].n_elec > 0.0 && tab[p].n_elec < (double)geo[p].n) || !(tab[p].beta > 0.0)) st = CHEBDM_ERR_ARG;
    else if (!(half > 0.0)) st = 2;
    else if (M < 0 || M > mcap || M < order + 1) st = CHEBDM_ERR_ARG;
    if (M < order + 1 || M > mcap) M = mcap;
    d.status = st;
    mq[p] = M;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_batch_shift(const BatchProblem* __restrict__ tab, const BatchGeom* __restrict__ geo,
              const DevScalars* __restrict__ s, T* __restrict__ mats) {
    const int p = blockIdx.z;
    const int64_t n = geo[p].n, ld = geo[p].ld;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const double cen = s[p].cen, half = s[p].half;
    const double* __restrict__ H = tab[p].H;
    const int64_t ldh = tab[p].ldh;
    T* __restrict__ out = mats + geo[p].off;
    for (int64_t i = blockIdx.y; i < n; i += gridDim.y) {   // rows i, i + gridDim.y, ...
        const double h = H[i * ldh + j];
        const double v = half > 0.0 ? (i == j ? h - cen : h) / half : 0.0;
        out[i * ld + j] = (T)v;
    }
}

// the last giant step writes the caller's D
template <typename T>
__global__ void k_batch_patch(const BatchProblem* __restrict__ tab, GemmDesc<T>* descs, int count) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= count) return;
    descs[p].Out = tab[p].D;
    descs[p].ld_out = tab[p].ldd;
}

// ---- moments: traces of T_1..T_k, Gram <T_{lk}, T_i>, assembly
template <typename T>
__global__ void __launch_bounds__(256)
k_batch_traces(const BatchGeom* __restrict__ geo, const T* __restrict__ mats, int k, double* __restrict__ trb) {
    __shared__ double smem[4];
    const int p = blockIdx.y, i = blockIdx.x;   // T_{i+1} in slot i
    const int64_t n = geo[p].n, ld = geo[p].ld;
    const T* a = mats + geo[p].off + (int64_t)i * ld * ld;
    double acc = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += 256) acc += (double)a[r * ld + r];
    acc = block_sum<256>(acc, smem);
    if (threadIdx.x == 0) trb[(int64_t)p * k + i] = acc;
}

// VW consecutive elements of one matrix per lane (32 bytes: 4 float64 or 8 float32), widened
// to float64, loaded as 16-byte vectors
template <int VW>
struct GLane {
    double v[VW];
};
template <int VW>
__device__ __forceinline__ GLane<VW> gload(const double* p) {   // one 32-byte vector load
    static_assert(VW == 4, "float64 lanes hold four elements");
    const f64x4 x = *reinterpret_cast<const f64x4*>(p);
    GLane<VW> out;
#pragma unroll
    for (int t = 0; t < 4; ++t) out.v[t] = x[t];
    return out;
}
template <int VW>
__device__ __forceinline__ GLane<VW> gload(const float* p) {    // one 32-byte vector load
    static_assert(VW == 8, "float32 lanes hold eight elements");
    typedef float f32x8v __attribute__((ext_vector_type(8)));
    const f32x8v x = *reinterpret_cast<const f32x8v*>(p);
    GLane<VW> out;
#pragma unroll
    for (int t = 0; t < 8; ++t) out.v[t] = (double)x[t];
    return out;
}

constexpr int kGM = 48;

// G[l][i] = <L_l, T_i>, L_1 = T_k (slot k-1), L_l = T_{lk} (slot k+l-2), T_i in slot i-1.
// Chunks of 4 VW elements: lane group lq holds VW consecutive elements of each of its matrices,
// so every (matrix, chunk) is one whole 128-byte line.
template <typename T, int FM, int FN, int VW = 32 / (int)sizeof(T)>
__global__ void __launch_bounds__(256)
k_batch_gram(const BatchGeom* __restrict__ geo, const T* __restrict__ mats, int k, int nl,
             double* __restrict__ partial) {
    __shared__ double red[FM * 16][FN * 16 + 1];
    const int p = blockIdx.y;
    const int64_t n = geo[p].n, ld = geo[p].ld, stride = ld * ld;
    const T* base = mats + geo[p].off;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lq = lane >> 4;
    constexpr int CH = 4 * VW;
    const int64_t nchunk = n * ld / CH;
    const int64_t gw = (int64_t)blockIdx.x * 4 + wave, nw = (int64_t)gridDim.x * 4;
    const int64_t c0 = nchunk * gw / nw, c1 = nchunk * (gw + 1) / nw;
    const T* pa[FM];
    const T* pb[FN];
#pragma unroll
    for (int f = 0; f < FM; ++f) {
        int l = f * 16 + lr + 1;                 // L index 1..nl
        if (l > nl) l = 1;
        const int64_t slot = (l == 1) ? k - 1 : k + l - 2;
        pa[f] = base + slot * stride + lq * VW;
    }
#pragma unroll
    for (int g = 0; g < FN; ++g) {
        int i = g * 16 + lr + 1;                 // T index 1..k
        if (i > k) i = 1;
        pb[g] = base + (int64_t)(i - 1) * stride + lq * VW;
    }
    f64x4 acc[FM][FN];
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int g = 0; g < FN; ++g) acc[f][g] = f64x4{0.0, 0.0, 0.0, 0.0};
    // two chunks per iteration: all their loads are issued before the first MFMA
    constexpr int U = 2;
    int64_t c = c0;
    for (; c + U <= c1; c += U) {
        GLane<VW> a[U][FM], b[U][FN];
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int f = 0; f < FM; ++f) a[u][f] = gload<VW>(pa[f] + (c + u) * CH);
#pragma unroll
            for (int g = 0; g < FN; ++g) b[u][g] = gload<VW>(pb[g] + (c + u) * CH);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int s = 0; s < VW; ++s)
#pragma unroll
                for (int f = 0; f < FM; ++f)
#pragma unroll
                    for (int g = 0; g < FN; ++g)
                        acc[f][g] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][f].v[s], b[u][g].v[s], acc[f][g], 0, 0, 0);
    }
    for (; c < c1; ++c) {
        const int64_t e = c * CH;
        GLane<VW> a[FM], b[FN];
#pragma unroll
        for (int f = 0; f < FM; ++f) a[f] = gload<VW>(pa[f] + e);
#pragma unroll
        for (int g = 0; g < FN; ++g) b[g] = gload<VW>(pb[g] + e);
#pragma unroll
        for (int s = 0; s < VW; ++s)
#pragma unroll
            for (int f = 0; f < FM; ++f)
#pragma unroll
                for (int g = 0; g < FN; ++g)
                    acc[f][g] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[f].v[s], b[g].v[s], acc[f][g], 0, 0, 0);
    }
    // float64 MFMA output: row lq + 4r, column lr of each 16 x 16 block; waves add in order
    for (int w = 0; w < 4; ++w) {
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
    double* out = partial + ((int64_t)p * gridDim.x + blockIdx.x) * kGM * kGM;
    for (int idx = threadIdx.x; idx < FM * 16 * FN * 16; idx += 256) {
        const int rr = idx / (FN * 16), cc = idx % (FN * 16);
        out[rr * kGM + cc] = red[rr][cc];
    }
}

// fold the Gram partials and assemble tau_0..tau_L (one work-group per problem)
__global__ void __launch_bounds__(64)
k_batch_tau(const BatchGeom* __restrict__ geo, const double* __restrict__ trb, const double* __restrict__ partial,
            int gram_blocks, int k, int m, int nl, int order, double* __restrict__ gram, double* __restrict__ tau) {
    const int p = blockIdx.x, tid = threadIdx.x;
    double* G = gram + (int64_t)p * kGM * kGM;
    for (int idx = tid; idx < nl * k; idx += 64) {
        const int l = idx / k, i = idx % k;
        double s = 0.0;
        for (int b = 0; b < gram_blocks; ++b) s += partial[((int64_t)p * gram_blocks + b) * kGM * kGM + l * kGM + i];
        G[l * k + i] = s;
    }
    double* t = tau + (int64_t)p * (order + 1);
    if (tid == 0) t[0] = (double)geo[p].n;
    for (int i = 1 + tid; i <= k && i <= order; i += 64) t[i] = trb[(int64_t)p * k + i - 1];
    __syncthreads();
    for (int l = 1; l < m; ++l) {
        for (int i = 1 + tid; i <= k; i += 64) {
            const int idx = l * k + i;
            if (idx <= order) t[idx] = 2.0 * G[(l - 1) * k + (i - 1)] - t[l * k - i];
        }
        __syncthreads();
    }
}

// ---- quadrature tables and the bisection
__global__ void __launch_bounds__(256)
k_batch_dct3(const double* __restrict__ tau, int order, const int64_t* __restrict__ mq, int64_t mcap,
             double* __restrict__ w, double* __restrict__ x, int damping) {
    extern __shared__ double st[];
    const int p = blockIdx.y;
    // the grid spans the largest quadrature the plan allows; work-groups past this problem's
    // M nodes (64 per work-group) leave at once, before staging the moments
    if ((int64_t)blockIdx.x * 64 >= mq[p]) return;
    for (int i = threadIdx.x; i <= order; i += 256)
        st[i] = tau[(int64_t)p * (order + 1) + i] * damping_factor(damping, i, order);
    __syncthreads();
    // four neighbouring lanes share node j, lane s summing n = s, s + 4, ... (as k_dct3)
    const int s = threadIdx.x & 3;
    const int64_t M = mq[p], j = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 2;
    const bool live = j < M;   // no early exit: every lane takes part in the shuffles
    const int64_t mod = 4 * M, q1 = 2 * j + 1, step = (4 * q1) % mod;
    double acc = 0.0;
    if (live) {
        int64_t q = (s * q1) % mod;
        for (int nn = s; nn <= order; nn += 4) {
            acc += nn == 0 ? st[0] : 2.0 * st[nn] * node_cos(q, M);
            q += step;
            if (q >= mod) q -= mod;
        }
    }
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    if (live && s == 0) {
        w[p * mcap + j] = acc;
        x[p * mcap + j] = node_cos(q1, M);
    }
}

constexpr int kBisect = 512;

// Chemical-potential search, one work-group per problem (modes as in search_dev.h; mode 2 takes
// the network's guess mu_hat[p]).
__global__ void __launch_bounds__(kBisect)
k_batch_search(const int64_t* __restrict__ mq, int64_t mcap, const double* __restrict__ w,
               const double* __restrict__ x, DevScalars* s, int mode, const float* __restrict__ mu_hat,
               double delta, double* __restrict__ scratch) {
    __shared__ double smem[kBisect / 64];
    const int p = blockIdx.x;
    DevScalars& d = s[p];
    if (d.status != 0) return;
    const double guess = mode == 2 ? (double)mu_hat[p] : 0.0;
    mu_search_one<kBisect>(mq[p], w + p * mcap, x + p * mcap, d, mode, guess, delta, smem, scratch + p * mcap);
}

// network inputs of problem p: tau_1..tau_62 / n, N_e / n, log(beta') / 4
__global__ void k_batch_features(const BatchGeom* __restrict__ geo, const double* __restrict__ tau, int order,
                                 const DevScalars* __restrict__ s, float* __restrict__ feat) {
    const int p = blockIdx.x, j = threadIdx.x;
    const double n = (double)geo[p].n;
    double v;
    if (j < 62) v = (j + 1 <= order) ? tau[(int64_t)p * (order + 1) + j + 1] / n : 0.0;
    else if (j == 62) v = s[p].n_elec / n;
    else v = log(s[p].beta_s > 0.0 ? s[p].beta_s : 1.0) / 4.0;
    feat[(int64_t)p * 64 + j] = (float)v;
}

// ---- coefficients at the found mu~ and the composition-form block coefficients
__global__ void __launch_bounds__(256)
k_batch_fermi(const int64_t* __restrict__ mq, int64_t mcap, const DevScalars* __restrict__ s, double* __restrict__ f) {
    const int p = blockIdx.y;
    const int64_t M = mq[p], j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= M) return;
    f[p * mcap + j] = fermi_scaled(node_cos(2 * j + 1, M), s[p].beta_s, s[p].mu_s);
}

__global__ void __launch_bounds__(256)
k_batch_dct2(const int64_t* __restrict__ mq, int64_t mcap, const double* __restrict__ f, int order,
             double* __restrict__ c, int damping) {
    __shared__ double smem[4];
    const int p = blockIdx.y;
    const int64_t n = blockIdx.x, M = mq[p], mod = 4 * M;
    const int64_t step = (512 * n) % mod;
    int64_t q = (n * (2 * (int64_t)threadIdx.x + 1)) % mod;
    const double* fp = f + p * mcap;
    double acc = 0.0;
    for (int64_t j = threadIdx.x; j < M; j += 256) {
        acc += fp[j] * node_cos(q, M);
        q += step;
        if (q >= mod) q -= mod;
    }
    acc = block_sum<256>(acc, smem);
    if (threadIdx.x == 0)
        c[(int64_t)p * (order + 1) + n] = (n == 0 ? 1.0 : 2.0) * acc / (double)M * damping_factor(damping, (int)n, order);
}

// e_{l,0} = c_{lk}; e_{l,i} = 2 c_{lk+i} - e_{l+1,k-i} (l >= 1); e_{0,i} = c_i - e_{1,k-i}/2
__global__ void __launch_bounds__(64)
k_batch_cform(const double* __restrict__ c, int order, int k, int m, double* __restrict__ coef) {
    __shared__ double e[kMaxBlocks][kMaxBlocks];
    const int p = blockIdx.x, tid = threadIdx.x;
    const double* cp = c + (int64_t)p * (order + 1);
    auto cpad = [&](int idx) -> double { return idx <= order ? cp[idx] : 0.0; };
    for (int l = m - 1; l >= 0; --l) {
        for (int i = tid; i < k; i += 64) {
            double v;
            if (i == 0) {
                v = cpad(l * k);
            } else {
                const double up = (l + 1 < m) ? e[l + 1][k - i] : 0.0;
                v = (l == 0) ? cpad(i) - 0.5 * up : 2.0 * cpad(l * k + i) - up;
            }
            e[l][i] = v;
        }
        __syncthreads();
    }
    for (int idx = tid; idx < k * m; idx += 64) coef[(int64_t)p * k * m + idx] = e[idx / k][idx % k];
}

// ---- block sums R_l = sum_i e_{l,i} T_i (T_0 = I), all l of a problem in one pass,
// 16-byte vectors along full padded rows (zero padding in, zero padding out)
template <typename T> struct BVec;
template <> struct BVec<double> { typedef double V __attribute__((ext_vector_type(2))); static constexpr int W = 2; };
template <> struct BVec<float> { typedef float V __attribute__((ext_vector_type(4))); static constexpr int W = 4; };

template <typename T, int MB>
__global__ void __launch_bounds__(256)
k_batch_combine(const BatchGeom* __restrict__ geo, const double* __restrict__ coef, int k, int m, int l0,
                T* __restrict__ mats) {
    using V = typename BVec<T>::V;
    constexpr int W = BVec<T>::W;
    const int p = blockIdx.z;
    const int64_t n = geo[p].n, ld = geo[p].ld, stride = ld * ld;
    const int64_t col = ((int64_t)blockIdx.x * 256 + threadIdx.x) * W;
    if (col >= ld) return;
    const T* tb = mats + geo[p].off;
    T* rb = mats + geo[p].off + (int64_t)k * stride;
    const double* cf = coef + (int64_t)p * k * m;
    const int lcount = (m - l0) < MB ? (m - l0) : MB;
    for (int64_t row = blockIdx.y; row < n; row += gridDim.y) {   // rows row, row + gridDim.y, ...
        const int64_t off = row * ld + col;
        double acc[MB][W];
#pragma unroll
        for (int l = 0; l < MB; ++l) {
            const double c0 = l < lcount ? cf[(int64_t)(l0 + l) * k] : 0.0;
#pragma unroll
            for (int w = 0; w < W; ++w) acc[l][w] = (col + w == row) ? c0 : 0.0;
        }
        for (int i = 1; i < k; ++i) {
            const V t = *reinterpret_cast<const V*>(tb + (int64_t)(i - 1) * stride + off);
#pragma unroll
            for (int l = 0; l < MB; ++l) {
                const double c = l < lcount ? cf[(int64_t)(l0 + l) * k + i] : 0.0;
#pragma unroll
                for (int w = 0; w < W; ++w) acc[l][w] += c * (double)t[w];
            }
        }
#pragma unroll
        for (int l = 0; l < MB; ++l) {
            if (l < lcount) {
                V o;
#pragma unroll
                for (int w = 0; w < W; ++w) o[w] = (T)acc[l][w];
                *reinterpret_cast<V*>(rb + (int64_t)(l0 + l) * stride + off) = o;
            }
        }
    }
}

// ---- results: tr D, mu, and D = (N_e/n) I for a scalar H
__global__ void __launch_bounds__(256)
k_batch_scalar_fill(const BatchProblem* __restrict__ tab, const BatchGeom* __restrict__ geo,
                    const DevScalars* __restrict__ s) {
    const int p = blockIdx.z;
    if (s[p].status != 2) return;
    const int64_t n = geo[p].n, j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    for (int64_t i = blockIdx.y; i < n; i += gridDim.y)
        tab[p].D[i * tab[p].ldd + j] = (i == j) ? tab[p].n_elec / (double)n : 0.0;
}

__global__ void __launch_bounds__(256)
k_batch_finish(const BatchProblem* __restrict__ tab, const BatchGeom* __restrict__ geo, DevScalars* s,
               double* __restrict__ mu, double* __restrict__ trD, int with_density) {
    __shared__ double smem[4];
    const int p = blockIdx.x;
    const int64_t n = geo[p].n;
    double acc = 0.0;
    if (with_density) {
        const double* D = tab[p].D;
        const int64_t ldd = tab[p].ldd;
        for (int64_t i = threadIdx.x; i < n; i += 256) acc += D[i * ldd + i];
        acc = block_sum<256>(acc, smem);
    } else {
        acc = s[p].status == 2 ? s[p].n_elec : s[p].trace;   // t(mu~) of the search
    }
    if (threadIdx.x == 0) {
        trD[p] = acc;
        DevScalars& d = s[p];
        if (d.status == 2) {   // H = cI: tr f(c) I = N_e fixes mu in closed form
            const double occ = d.n_elec / (double)n;
            mu[p] = d.emin - log(1.0 / occ - 1.0) / tab[p].beta;
            d.trace = d.n_elec;
            d.status = CHEBDM_OK;
        } else {
            mu[p] = d.cen + d.half * d.mu_s;
        }
    }
}

// Row groups of the per-row kernels (shift, combine, scalar fill): work-group y takes rows
// y, y + G, ... of its problem, so a problem smaller than the largest launches no idle
// work-groups (one work-group per row of the largest problem cost 0.9 ms per 512-problem
// batch in the fill alone, which has work only for a scalar H).
inline int batch_row_groups(int64_t nmax) { return nmax < 64 ? (int)nmax : 64; }

template <typename T>
hipError_t combine_all(const BatchDims& d, const BatchGeom* geo, const double* coef, T* mats, hipStream_t st) {
    const int64_t per = 256 * BVec<T>::W;
    dim3 grid((unsigned)((d.ldmax + per - 1) / per), (unsigned)batch_row_groups(d.nmax), (unsigned)d.count);
    for (int l0 = 0; l0 < d.m; l0 += 24) {
        const int cnt = (d.m - l0) < 24 ? (d.m - l0) : 24;
        if (cnt <= 8)
            hipLaunchKernelGGL((k_batch_combine<T, 8>), grid, dim3(256), 0, st, geo, coef, d.k, d.m, l0, mats);
        else if (cnt <= 16)
            hipLaunchKernelGGL((k_batch_combine<T, 16>), grid, dim3(256), 0, st, geo, coef, d.k, d.m, l0, mats);
        else
            hipLaunchKernelGGL((k_batch_combine<T, 24>), grid, dim3(256), 0, st, geo, coef, d.k, d.m, l0, mats);
    }
    return hipGetLastError();
}

template <typename T, int FM>
void gram_fm(int fn, dim3 grid, const BatchGeom* geo, const T* mats, int k, int nl, double* partial, hipStream_t st) {
    if (fn == 1) hipLaunchKernelGGL((k_batch_gram<T, FM, 1>), grid, dim3(256), 0, st, geo, mats, k, nl, partial);
    else if (fn == 2) hipLaunchKernelGGL((k_batch_gram<T, FM, 2>), grid, dim3(256), 0, st, geo, mats, k, nl, partial);
    else hipLaunchKernelGGL((k_batch_gram<T, FM, 3>), grid, dim3(256), 0, st, geo, mats, k, nl, partial);
}

template <typename T>
hipError_t moments_t(const BatchDims& d, const BatchGeom* geo, const T* mats, double* trb, double* partial,
                     int gram_blocks, double* gram, double* tau, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_traces<T>, dim3((unsigned)d.k, (unsigned)d.count), dim3(256), 0, st, geo, mats, d.k,
                       trb);
    if (d.lmax >= 1) {
        dim3 grid((unsigned)gram_blocks, (unsigned)d.count);
        const int fm = (d.lmax + 15) / 16, fn = (d.k + 15) / 16;
        if (fm == 1) gram_fm<T, 1>(fn, grid, geo, mats, d.k, d.lmax, partial, st);
        else if (fm == 2) gram_fm<T, 2>(fn, grid, geo, mats, d.k, d.lmax, partial, st);
        else gram_fm<T, 3>(fn, grid, geo, mats, d.k, d.lmax, partial, st);
    }
    hipLaunchKernelGGL(k_batch_tau, dim3((unsigned)d.count), dim3(64), 0, st, geo, (const double*)trb,
                       (const double*)partial, d.lmax >= 1 ? gram_blocks : 0, d.k, d.m, d.lmax, d.order, gram, tau);
    return hipGetLastError();
}

}  // namespace

int batch_gemm_grid(int prec) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1024;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1024;
    hipError_t e = hipSuccess;
    switch (prec) {
        case CHEBDM_FP64: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch_gemm<P_F64>, 64, 0); break;
        case CHEBDM_FP32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch_gemm<P_F32>, 64, 0); break;
        case CHEBDM_BF16X3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch_gemm<P_BF16X3>, 64, 0); break;
        default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch_gemm<P_BF16X6>, 64, 0); break;
    }
    if (e != hipSuccess || per < 1) per = 4;
    return cus * per;
}

hipError_t launch_batch_gemm(int prec, const void* descs, const BatchGeom* geo, const TileItem* items, int nitems,
                             int* counter, int grid, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    if (grid > nitems) grid = nitems;
    switch (prec) {
        case CHEBDM_FP64:
            hipLaunchKernelGGL(k_batch_gemm<P_F64>, dim3(grid), dim3(64), 0, st, (const GemmDesc<double>*)descs, geo,
                               items, nitems, counter);
            break;
        case CHEBDM_FP32:
            hipLaunchKernelGGL(k_batch_gemm<P_F32>, dim3(grid), dim3(64), 0, st, (const GemmDesc<float>*)descs, geo,
                               items, nitems, counter);
            break;
        case CHEBDM_BF16X3:
            hipLaunchKernelGGL(k_batch_gemm<P_BF16X3>, dim3(grid), dim3(64), 0, st, (const GemmDesc<float>*)descs,
                               geo, items, nitems, counter);
            break;
        default:
            hipLaunchKernelGGL(k_batch_gemm<P_BF16X6>, dim3(grid), dim3(64), 0, st, (const GemmDesc<float>*)descs,
                               geo, items, nitems, counter);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_batch_zero(int* p, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_batch_bounds(const BatchDims& d, const BatchProblem* tab, const BatchGeom* geo, double* colsum,
                               DevScalars* s, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_colsum, dim3((unsigned)((d.nmax + 255) / 256), (unsigned)d.count), dim3(256), 0, st, tab,
                       geo, colsum);
    hipLaunchKernelGGL(k_batch_bounds_final, dim3((unsigned)d.count), dim3(256), 0, st, tab, geo,
                       (const double*)colsum, s);
    return hipGetLastError();
}

hipError_t launch_batch_setup(const BatchDims& d, const BatchProblem* tab, const BatchGeom* geo, DevScalars* s,
                              int64_t* mq, double tol, int max_iter, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_setup, dim3((unsigned)((d.count + 63) / 64)), dim3(64), 0, st, tab, geo, s, mq, d.count,
                       d.order, d.mcap, tol, max_iter);
    return hipGetLastError();
}

hipError_t launch_batch_shift(const BatchDims& d, const BatchProblem* tab, const BatchGeom* geo, const DevScalars* s,
                              void* mats, hipStream_t st) {
    dim3 grid((unsigned)((d.nmax + 255) / 256), (unsigned)batch_row_groups(d.nmax), (unsigned)d.count);
    if (d.prec == CHEBDM_FP64)
        hipLaunchKernelGGL(k_batch_shift<double>, grid, dim3(256), 0, st, tab, geo, s, (double*)mats);
    else
        hipLaunchKernelGGL(k_batch_shift<float>, grid, dim3(256), 0, st, tab, geo, s, (float*)mats);
    return hipGetLastError();
}

hipError_t launch_batch_patch(const BatchDims& d, const BatchProblem* tab, void* final_descs, hipStream_t st) {
    dim3 grid((unsigned)((d.count + 63) / 64));
    if (d.prec == CHEBDM_FP64)
        hipLaunchKernelGGL(k_batch_patch<double>, grid, dim3(64), 0, st, tab, (GemmDesc<double>*)final_descs, d.count);
    else
        hipLaunchKernelGGL(k_batch_patch<float>, grid, dim3(64), 0, st, tab, (GemmDesc<float>*)final_descs, d.count);
    return hipGetLastError();
}

hipError_t launch_batch_moments(const BatchDims& d, const BatchGeom* geo, const void* mats, double* trb,
                                double* partial, int gram_blocks, double* gram, double* tau, hipStream_t st) {
    if (d.k > kGM || d.lmax > kGM) return hipErrorInvalidValue;
    if (d.prec == CHEBDM_FP64)
        return moments_t<double>(d, geo, (const double*)mats, trb, partial, gram_blocks, gram, tau, st);
    return moments_t<float>(d, geo, (const float*)mats, trb, partial, gram_blocks, gram, tau, st);
}

hipError_t launch_batch_search(const BatchDims& d, const double* tau, const int64_t* mq, double* w, double* x,
                               DevScalars* s, int mode, const float* mu_hat, double delta, double* scratch,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_batch_dct3, dim3((unsigned)((4 * d.mcap + 255) / 256), (unsigned)d.count), dim3(256),
                       sizeof(double) * (size_t)(d.order + 1), st, tau, d.order, mq, d.mcap, w, x, d.damping);
    hipLaunchKernelGGL(k_batch_search, dim3((unsigned)d.count), dim3(kBisect), 0, st, mq, d.mcap, (const double*)w,
                       (const double*)x, s, mode, mu_hat, delta, scratch);
    return hipGetLastError();
}

hipError_t launch_batch_features(const BatchDims& d, const BatchGeom* geo, const double* tau, const DevScalars* s,
                                 float* feat, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_features, dim3((unsigned)d.count), dim3(64), 0, st, geo, tau, d.order, s, feat);
    return hipGetLastError();
}

hipError_t launch_batch_coeffs(const BatchDims& d, const int64_t* mq, const DevScalars* s, double* ftab, double* c,
                               double* coef, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_fermi, dim3((unsigned)((d.mcap + 255) / 256), (unsigned)d.count), dim3(256), 0, st, mq,
                       d.mcap, s, ftab);
    hipLaunchKernelGGL(k_batch_dct2, dim3((unsigned)(d.order + 1), (unsigned)d.count), dim3(256), 0, st, mq, d.mcap,
                       (const double*)ftab, d.order, c, d.damping);
    hipLaunchKernelGGL(k_batch_cform, dim3((unsigned)d.count), dim3(64), 0, st, (const double*)c, d.order, d.k, d.m,
                       coef);
    return hipGetLastError();
}

hipError_t launch_batch_combine(const BatchDims& d, const BatchGeom* geo, const double* coef, void* mats,
                                hipStream_t st) {
    if (d.prec == CHEBDM_FP64) return combine_all<double>(d, geo, coef, (double*)mats, st);
    return combine_all<float>(d, geo, coef, (float*)mats, st);
}

hipError_t launch_batch_finish(const BatchDims& d, const BatchProblem* tab, const BatchGeom* geo, DevScalars* s,
                               double* mu, double* trD, int with_density, hipStream_t st) {
    if (with_density)
        hipLaunchKernelGGL(k_batch_scalar_fill, dim3((unsigned)((d.nmax + 255) / 256),
                                                     (unsigned)batch_row_groups(d.nmax), (unsigned)d.count),
                           dim3(256), 0, st, tab, geo, (const DevScalars*)s);
    hipLaunchKernelGGL(k_batch_finish, dim3((unsigned)d.count), dim3(256), 0, st, tab, geo, s, mu, trD, with_density);
    return hipGetLastError();
}

}  // namespace chebdm
