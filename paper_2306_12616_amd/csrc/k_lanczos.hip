// Tight spectral bounds by a few Lanczos steps (an alternative to Gershgorin's
// discs for the extreme eigenvalues e_a, e_b of Sec. II.B, which the paper
// asks for without naming a method).
//
// Start vector: SplitMix64 (Steele, Lea, Flood 2014) doubles in [-1, 1),
// normalised.  Step j (0-based), with one full reorthogonalisation pass:
//     w = H v_j;  alpha_j = v_j . w;  w -= alpha_j v_j + beta_{j-1} v_{j-1};
//     w -= sum_{i<=j} (v_i . w) v_i;   beta_j = ||w||;   v_{j+1} = w / beta_j.
// The recurrence ends after `steps` steps or when beta_j falls to 1e-12 times
// the Gershgorin scale max(|g_lo|, |g_hi|) (an invariant subspace).  The bounds
// are [theta_min - r, theta_max + r] with theta the extreme eigenvalues of the
// tridiagonal T_k and r = beta_{k-1}, widened by margin * width on each side
// and intersected with the Gershgorin interval already in the scalars (the
// Gershgorin interval alone if the intersection is empty).
//
// Kernels per step: the product H v_j (one wavefront per two rows, H read once
// along rows), alpha (one work-group; folded into the next kernel up to n = 8192),
// the three-term update with the partial projections v_i . w (a grid of slices
// x (j + 1)), and the reorthogonalisation with the partial norm.  Every reduction is a fixed-order sum of per-block
// partials, so the result does not depend on scheduling.  The tridiagonal
// extremes come from Sturm-sequence multisection (Barth, Martin, Wilkinson 1967)
// in one work-group.
//
// The same kernels serve one problem and a batch of problems of different n
// (the batched form): blockIdx.y (blockIdx.z for the projections) selects the
// problem, whose workspace, scalars and step count min(steps, n) are its own.
#include <cmath>

#include "internal.h"
#include "reduce.h"

namespace chebdm {

namespace {

constexpr int kNT = 256;
constexpr int kSlice = 1024;       // vector elements per work-group (4 per thread)
constexpr int kRowsPerWave = 2;
constexpr int kRowsPerBlock = (kNT / 64) * kRowsPerWave;
constexpr double kBreakdown = 1e-12;

__host__ __device__ inline int64_t blocks_of(int64_t n, int64_t per) { return (n + per - 1) / per; }

// One problem of a run: its matrix, size, scalars, workspace views and step count.
struct LzProblem {
    const double* H;
    int64_t n, ldh;
    DevScalars* s;
    LanczosWork L;
    int k, nbv, nbr;
};

__device__ inline LzProblem problem_of(const LanczosRun& r, int p) {
    LzProblem q;
    if (r.tab) {
        q.H = r.tab[p].H;
        q.ldh = r.tab[p].ldh;
        q.n = r.geo[p].n;
    } else {
        q.H = r.H;
        q.ldh = r.ldh;
        q.n = r.n;
    }
    q.s = r.s + p;
    q.k = (int)(q.n < r.steps ? q.n : r.steps);
    q.L = lanczos_layout(r.base + (int64_t)p * r.stride, q.n, q.k);
    q.nbv = (int)blocks_of(q.n, kSlice);
    q.nbr = (int)blocks_of(q.n, kRowsPerBlock);
    return q;
}

__device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Fixed-order sum of count partials by one work-group (every thread gets it).
__device__ inline double sum_partials(const double* __restrict__ p, int count, double* smem) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < count; b += kNT) acc += p[b];
    return block_sum<kNT>(acc, smem);
}

__global__ void __launch_bounds__(kNT) k_lz_init(const LanczosRun r) {
    __shared__ double smem[kNT / 64];
    const LzProblem q = problem_of(r, blockIdx.y);
    if ((int)blockIdx.x >= q.nbv) return;
    const int64_t base = (int64_t)blockIdx.x * kSlice;
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < kSlice / kNT; ++c) {
        const int64_t e = base + c * kNT + threadIdx.x;
        if (e < q.n) {
            const uint64_t z = splitmix64_at(r.seed, (uint64_t)e);
            const double u = 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
            q.L.w[e] = u;
            acc += u * u;
        }
    }
    acc = block_sum<kNT>(acc, smem);
    if (threadIdx.x == 0) q.L.pn[blockIdx.x] = acc;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        q.L.state[0] = 0;   // steps done at a breakdown (0: none)
        q.L.state[1] = 0;   // steps done in total
    }
}

// beta = ||w|| from the partial norms; v_j = w / beta; w2 = (H w) / beta; partial v_j . w2.
__global__ void __launch_bounds__(kNT) k_lz_matvec(const LanczosRun r, int j) {
    __shared__ double smem[kNT / 64];
    __shared__ double part[kNT / 64];
    const LzProblem q = problem_of(r, blockIdx.y);
    if (j >= q.k || (int)blockIdx.x >= q.nbr || q.L.state[0]) return;
    const int64_t n = q.n;
    const double bt = sqrt(sum_partials(q.L.pn, q.nbv, smem));
    if (j > 0) {
        const double scale = fmax(fabs(q.s->emin), fabs(q.s->emax));
        const bool broke = !(bt > kBreakdown * scale);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            q.L.beta[j - 1] = bt;
            if (broke) q.L.state[0] = j;
        }
        if (broke) return;
    }
    const double* __restrict__ w = q.L.w;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t r0 = (int64_t)blockIdx.x * kRowsPerBlock + wave * kRowsPerWave;
    double y[kRowsPerWave];
#pragma unroll
    for (int t = 0; t < kRowsPerWave; ++t) y[t] = 0.0;
    if (r0 < n) {
        const double* h0 = q.H + r0 * q.ldh;
        const double* h1 = q.H + (r0 + 1 < n ? r0 + 1 : r0) * q.ldh;
#pragma unroll 4
        for (int64_t c = lane; c < n; c += 64) {
            const double x = w[c];
            y[0] = fma(h0[c], x, y[0]);
            y[1] = fma(h1[c], x, y[1]);
        }
    }
#pragma unroll
    for (int t = 0; t < kRowsPerWave; ++t) y[t] = wave_sum(y[t]);
    if (lane == 0) {
        double contrib = 0.0;
#pragma unroll
        for (int t = 0; t < kRowsPerWave; ++t) {
            const int64_t row = r0 + t;
            if (row < n) {
                const double v = w[row] / bt;
                const double z = y[t] / bt;
                q.L.V[(int64_t)j * n + row] = v;
                q.L.w2[row] = z;
                contrib += v * z;
            }
        }
        part[wave] = contrib;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < kNT / 64; ++c) acc += part[c];
        q.L.pa[blockIdx.x] = acc;
    }
}

__global__ void __launch_bounds__(kNT) k_lz_alpha(const LanczosRun r, int j) {
    __shared__ double smem[kNT / 64];
    const LzProblem q = problem_of(r, blockIdx.y);
    if (j >= q.k || q.L.state[0]) return;
    const double a = sum_partials(q.L.pa, q.nbr, smem);
    if (threadIdx.x == 0) q.L.alpha[j] = a;
}

// x = w2 - alpha_j v_j - beta_{j-1} v_{j-1} on a slice (stored by the blockIdx.y == 0 row
// of blocks); partial v_i . x for i = blockIdx.y.  With fuse_alpha every block folds the
// alpha partials itself (the same fixed order as k_lz_alpha) and block (0, 0) stores alpha_j.
__global__ void __launch_bounds__(kNT) k_lz_proj(const LanczosRun r, int j, int fuse_alpha) {
    __shared__ double smem[kNT / 64];
    const LzProblem q = problem_of(r, blockIdx.z);
    if (j >= q.k || (int)blockIdx.x >= q.nbv || q.L.state[0]) return;
    const int64_t n = q.n;
    const int i = blockIdx.y;
    double a;
    if (fuse_alpha) {
        a = sum_partials(q.L.pa, q.nbr, smem);
        if (blockIdx.x == 0 && i == 0 && threadIdx.x == 0) q.L.alpha[j] = a;
    } else {
        a = q.L.alpha[j];
    }
    const double bm = j > 0 ? q.L.beta[j - 1] : 0.0;
    const double* vj = q.L.V + (int64_t)j * n;
    const double* vm = q.L.V + (int64_t)(j > 0 ? j - 1 : 0) * n;
    const double* vi = q.L.V + (int64_t)i * n;
    const int64_t base = (int64_t)blockIdx.x * kSlice;
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < kSlice / kNT; ++c) {
        const int64_t e = base + c * kNT + threadIdx.x;
        if (e < n) {
            double x = q.L.w2[e] - a * vj[e];
            if (j > 0) x -= bm * vm[e];
            if (i == 0) q.L.w[e] = x;
            acc += vi[e] * x;
        }
    }
    acc = block_sum<kNT>(acc, smem);
    if (threadIdx.x == 0) q.L.pc[(int64_t)i * q.nbv + blockIdx.x] = acc;
}

// c_i = sum of the partials; w -= sum_{i<=j} c_i v_i on a slice; partial ||w||^2.
__global__ void __launch_bounds__(kNT) k_lz_reorth(const LanczosRun r, int j) {
    __shared__ double smem[kNT / 64];
    __shared__ double c[kMaxLanczosSteps];
    const LzProblem q = problem_of(r, blockIdx.y);
    if (j >= q.k || (int)blockIdx.x >= q.nbv || q.L.state[0]) return;
    const int64_t n = q.n;
    for (int i = threadIdx.x; i <= j; i += kNT) {
        double acc = 0.0;
        for (int b = 0; b < q.nbv; ++b) acc += q.L.pc[(int64_t)i * q.nbv + b];
        c[i] = acc;
    }
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSlice;
    double acc = 0.0;
#pragma unroll
    for (int t = 0; t < kSlice / kNT; ++t) {
        const int64_t e = base + t * kNT + threadIdx.x;
        if (e < n) {
            double x = q.L.w[e];
            for (int i = 0; i <= j; ++i) x -= c[i] * q.L.V[(int64_t)i * n + e];
            q.L.w[e] = x;
            acc += x * x;
        }
    }
    acc = block_sum<kNT>(acc, smem);
    if (threadIdx.x == 0) q.L.pn[blockIdx.x] = acc;
}

// Number of eigenvalues of the tridiagonal (a, b) below x (Sturm sequence of the LDL^T pivots).
__device__ inline int sturm_count(const double* a, const double* b, int k, double x) {
    constexpr double pivmin = 1e-300;
    int cnt = 0;
    double q = a[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
    for (int i = 1; i < k; ++i) {
        q = (a[i] - x) - b[i - 1] * b[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += q < 0.0;
    }
    return cnt;
}

constexpr int kFinalNT = 128;   // wave 0: theta_min, wave 1: theta_max
constexpr int kRounds = 12;     // 65-way multisection: 65^12 > 2^72

__global__ void __launch_bounds__(kFinalNT) k_lz_final(const LanczosRun r) {
    __shared__ double a[kMaxLanczosSteps], b[kMaxLanczosSteps];
    __shared__ double theta[2];
    __shared__ double smem[kFinalNT / 64];
    __shared__ double r_last;
    const LzProblem q = problem_of(r, blockIdx.y);
    const int done = q.L.state[0];
    const int k = done ? done : q.k;
    double acc = 0.0;
    for (int c = threadIdx.x; c < q.nbv; c += kFinalNT) acc += q.L.pn[c];
    acc = block_sum<kFinalNT>(acc, smem);
    if (threadIdx.x == 0) {
        r_last = done ? q.L.beta[k - 1] : sqrt(acc);
        if (!done) q.L.beta[k - 1] = r_last;
        q.L.state[1] = k;
    }
    for (int i = threadIdx.x; i < k; i += kFinalNT) {
        a[i] = q.L.alpha[i];
        b[i] = i + 1 < k ? q.L.beta[i] : 0.0;
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // Gershgorin interval of T
    double lo = INFINITY, hi = -INFINITY;
    for (int i = 0; i < k; ++i) {
        const double rad = fabs(b[i]) + (i > 0 ? fabs(b[i - 1]) : 0.0);
        lo = fmin(lo, a[i] - rad);
        hi = fmax(hi, a[i] + rad);
    }
    // wave 0: smallest x with count(x) >= 1 (theta_min in [lo, hi]); wave 1: count(x) >= k
    const int need = wave == 0 ? 1 : k;
    for (int round = 0; round < kRounds; ++round) {
        const double x = lo + (hi - lo) * (double)(lane + 1) / 65.0;
        const bool ge = sturm_count(a, b, k, x) >= need;
        const uint64_t mask = __ballot(ge);
        const int first = mask ? __ffsll((unsigned long long)mask) - 1 : 64;
        const double xl = first == 0 ? lo : lo + (hi - lo) * (double)first / 65.0;
        const double xh = first == 64 ? hi : lo + (hi - lo) * (double)(first + 1) / 65.0;
        lo = xl;
        hi = xh;
    }
    if (lane == 0) theta[wave] = wave == 0 ? lo : hi;   // outer side of the final interval
    __syncthreads();
    if (threadIdx.x == 0) {
        const double g_lo = q.s->emin, g_hi = q.s->emax;
        double e_lo = theta[0] - r_last, e_hi = theta[1] + r_last;
        const double pad = r.margin * (e_hi - e_lo);
        e_lo = fmax(e_lo - pad, g_lo);
        e_hi = fmin(e_hi + pad, g_hi);
        if (!(e_lo <= e_hi)) {
            e_lo = g_lo;
            e_hi = g_hi;
        }
        q.s->emin = e_lo;
        q.s->emax = e_hi;
    }
}

}  // namespace

int64_t lanczos_work_doubles(int64_t n, int steps) {
    const int64_t nbv = blocks_of(n, kSlice), nbr = blocks_of(n, kRowsPerBlock);
    return (int64_t)steps * n + 2 * n + nbr + (int64_t)steps * nbv + nbv + 2 * (int64_t)steps + 2;
}

__host__ __device__ LanczosWork lanczos_layout(double* base, int64_t n, int steps) {
    const int64_t nbv = blocks_of(n, kSlice), nbr = blocks_of(n, kRowsPerBlock);
    LanczosWork L;
    double* p = base;
    L.V = p;
    p += (int64_t)steps * n;
    L.w = p;
    p += n;
    L.w2 = p;
    p += n;
    L.pa = p;
    p += nbr;
    L.pc = p;
    p += (int64_t)steps * nbv;
    L.pn = p;
    p += nbv;
    L.alpha = p;
    p += steps;
    L.beta = p;
    p += steps;
    L.state = reinterpret_cast<int32_t*>(p);   // two int32 in one double
    return L;
}

hipError_t launch_lanczos_run(const LanczosRun& r, int count, hipStream_t st) {
    if (r.steps < 1 || r.steps > kMaxLanczosSteps || count < 1 || count > 65535 || r.nmax < 1) return hipErrorInvalidValue;
    if (r.stride < lanczos_work_doubles(r.nmax, r.steps)) return hipErrorInvalidValue;
    const int nbv = (int)blocks_of(r.nmax, kSlice), nbr = (int)blocks_of(r.nmax, kRowsPerBlock);
    const int steps = (int)(r.nmax < r.steps ? r.nmax : r.steps);
    // up to 1024 alpha partials (n <= 8192) every projection block folds them itself: one
    // launch per step fewer; beyond that one work-group folds them once
    const int fuse = nbr <= 1024 ? 1 : 0;
    hipLaunchKernelGGL(k_lz_init, dim3(nbv, count), dim3(kNT), 0, st, r);
    for (int j = 0; j < steps; ++j) {
        hipLaunchKernelGGL(k_lz_matvec, dim3(nbr, count), dim3(kNT), 0, st, r, j);
        if (!fuse) hipLaunchKernelGGL(k_lz_alpha, dim3(1, count), dim3(kNT), 0, st, r, j);
        hipLaunchKernelGGL(k_lz_proj, dim3(nbv, j + 1, count), dim3(kNT), 0, st, r, j, fuse);
        hipLaunchKernelGGL(k_lz_reorth, dim3(nbv, count), dim3(kNT), 0, st, r, j);
    }
    hipLaunchKernelGGL(k_lz_final, dim3(1, count), dim3(kFinalNT), 0, st, r);
    return hipGetLastError();
}

hipError_t launch_lanczos(const double* H, int64_t n, int64_t ldh, int steps, double margin, uint64_t seed,
                          double* work, DevScalars* s, hipStream_t st) {
    if (steps < 1 || steps > kMaxLanczosSteps || steps > n) return hipErrorInvalidValue;
    LanczosRun r{};
    r.H = H;
    r.n = n;
    r.ldh = ldh;
    r.s = s;
    r.base = work;
    r.stride = lanczos_work_doubles(n, steps);
    r.nmax = n;
    r.steps = steps;
    r.margin = margin;
    r.seed = seed;
    return launch_lanczos_run(r, 1, st);
}

}  // namespace chebdm
