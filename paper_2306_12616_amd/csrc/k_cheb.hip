// Scalar side of the method on the device, all in float64:
//   - Chebyshev coefficients of the Fermi function (expansion sum c_n T_n,
//     Sec. II.B; obtained by a Chebyshev-Gauss projection, i.e. a DCT-II);
//   - block coefficients: the paper's power form d (eqs. "formula for d0",
//     "formula for d", "X": back substitution over row blocks) or the
//     composition form e (same identity 2 T_a T_b = T_{a+b} + T_{|a-b|});
//   - trace moments tau_n from traces and Gram products of Chebyshev matrices;
//   - the chemical-potential bisection on t(mu~) = sum_n c_n(mu~) tau_n,
//     rewritten as (1/M) sum_j f(x_j; mu~) w_j with w the DCT-III of tau.
// Angles are reduced exactly in integers: cos(n theta_j) = cospi(q / 2M)
// with q = n (2j+1) mod 4M, so every cosine is a correctly reduced cospi.
#include <cmath>

#include "cheb_dev.h"
#include "internal.h"
#include "reduce.h"
#include "search_dev.h"

namespace chebdm {

namespace {

// bounds_on_device: take e_a, e_b from s (written there by the Gershgorin kernels) instead of
// the arguments, so that a captured graph does not depend on their values.
__global__ void k_set_scalars(DevScalars* s, double emin, double emax, double beta, double mu,
                              int has_mu, double n_elec, double tol, int max_iter, int bounds_on_device) {
    if (bounds_on_device) {
        emin = s->emin;
        emax = s->emax;
    }
    const double cen = 0.5 * (emin + emax), half = 0.5 * (emax - emin);
    s->emin = emin;
    s->emax = emax;
    s->cen = cen;
    s->half = half;
    s->beta_s = beta * half;
    s->mu_s = has_mu ? (mu - cen) / half : 0.0;
    s->n_elec = n_elec;
    s->tol = tol;
    s->max_iter = max_iter;
    s->status = 0;
    s->iters = 0;
    s->trace = 0.0;
}

__global__ void __launch_bounds__(256)
k_fermi_table(int64_t M, const DevScalars* __restrict__ s, double* __restrict__ f) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= M) return;
    const double x = node_cos(2 * j + 1, M);
    f[j] = fermi_scaled(x, s->beta_s, s->mu_s);
}

// One workgroup per coefficient n: c_n = (2 - delta_{n0})/M sum_j f_j cos(n theta_j).
__global__ void __launch_bounds__(256)
k_dct2(int64_t M, const double* __restrict__ f, double* __restrict__ c, int order, int damping) {
    __shared__ double smem[4];
    const int64_t n = blockIdx.x;
    const int64_t mod = 4 * M;
    // q_j = n (2j+1) mod 4M, advanced by 2n*256 per stride without a 64-bit divide
    const int64_t step = (512 * n) % mod;
    int64_t q = (n * (2 * (int64_t)threadIdx.x + 1)) % mod;
    double acc = 0.0;
    for (int64_t j = threadIdx.x; j < M; j += 256) {
        acc += f[j] * node_cos(q, M);
        q += step;
        if (q >= mod) q -= mod;
    }
    acc = block_sum<256>(acc, smem);
    if (threadIdx.x == 0) c[n] = (n == 0 ? 1.0 : 2.0) * acc / (double)M * damping_factor(damping, (int)n, order);
}

// Block coefficients, one workgroup.  Output coef[l*k + i] = weight of T_i in block l.
__global__ void __launch_bounds__(64)
k_block_coeffs(const double* __restrict__ c, int order, int k, int m, int form,
               double* __restrict__ coef) {
    __shared__ double a[kMaxBlocks][kMaxBlocks];   // a[j][l] of T_k^j = sum_l a_{j,l} T_{lk}
    __shared__ double d[kMaxBlocks][kMaxBlocks];   // d[l][i]: block l, index i (output layout)
    const int tid = threadIdx.x;
    auto cpad = [&](int idx) -> double { return idx <= order ? c[idx] : 0.0; };

    if (form == CHEBDM_GIANT_COMPOSITION) {
        // e_{l,0} = c_{lk}; e_{l,i} = 2 c_{lk+i} - e_{l+1,k-i} (l >= 1); e_{0,i} = c_i - e_{1,k-i}/2
        for (int l = m - 1; l >= 0; --l) {
            for (int i = tid; i < k; i += blockDim.x) {
                double v;
                if (i == 0) {
                    v = cpad(l * k);
                } else {
                    const double up = (l + 1 < m) ? d[l + 1][k - i] : 0.0;
                    v = (l == 0) ? cpad(i) - 0.5 * up : 2.0 * cpad(l * k + i) - up;
                }
                d[l][i] = v;
            }
            __syncthreads();
        }
    } else {
        // Matrix A by the recurrence of eq. "coeff recursion" (row j from row j-1).
        for (int l = tid; l < m; l += blockDim.x)
            for (int j = 0; j < m; ++j) a[j][l] = 0.0;
        __syncthreads();
        if (tid == 0) {
            a[0][0] = 1.0;
            if (m > 1) a[1][1] = 1.0;
        }
        __syncthreads();
        for (int j = 2; j < m; ++j) {
            for (int l = tid; l <= j; l += blockDim.x) {
                auto prev = [&](int ll) -> double { return (ll >= 0 && ll <= j - 1) ? a[j - 1][ll] : 0.0; };
                double v;
                if (l == 0) v = 0.5 * prev(1);
                else if (l == 1) v = prev(0) + 0.5 * prev(2);
                else if (l < j) v = 0.5 * (prev(l - 1) + prev(l + 1));
                else v = 0.5 * prev(l - 1);
                a[j][l] = v;
            }
            __syncthreads();
        }
        // Back substitution over the row blocks of X, l = m-1 down to 0.  Row
        // (l, i) involves d_{i,j} for j >= l and d_{k-i,j} for j >= l+1 only.
        for (int l = m - 1; l >= 0; --l) {
            for (int i = tid; i < k; i += blockDim.x) {
                double s = cpad(l * k + i);
                double v;
                if (i == 0) {
                    for (int j = l + 1; j < m; ++j) s -= a[j][l] * d[j][0];
                    v = s / a[l][l];
                } else {
                    const double own = (l == 0) ? 1.0 : 0.5;
                    double t = 0.0;
                    for (int j = l + 1; j < m; ++j) t += a[j][l] * d[j][i];
                    s -= own * t;
                    if (l + 1 < m) {
                        double u = 0.0;
                        for (int j = l + 1; j < m; ++j) u += a[j][l + 1] * d[j][k - i];
                        s -= 0.5 * u;
                    }
                    v = s / (own * a[l][l]);
                }
                d[l][i] = v;
            }
            __syncthreads();
        }
    }
    for (int idx = tid; idx < k * m; idx += blockDim.x) coef[idx] = d[idx / k][idx % k];
}

// tau_0 = n, tau_i = tr T_i (i <= k), tau_{lk+i} = 2 <T_{lk}, T_i> - tau_{lk-i}.
__global__ void __launch_bounds__(64)
k_assemble_moments(const double* __restrict__ tr_baby, const double* __restrict__ gram, int k, int m,
                   int order, int64_t n, double* __restrict__ tau) {
    const int tid = threadIdx.x;
    if (tid == 0) tau[0] = (double)n;
    for (int i = 1 + tid; i <= k && i <= order; i += blockDim.x) tau[i] = tr_baby[i - 1];
    __syncthreads();
    for (int l = 1; l < m; ++l) {
        for (int i = 1 + tid; i <= k; i += blockDim.x) {
            const int idx = l * k + i;
            if (idx <= order) tau[idx] = 2.0 * gram[(l - 1) * k + (i - 1)] - tau[l * k - i];
        }
        __syncthreads();
    }
}

// w_j = sum_n (2 - delta_{n0}) tau_n cos(n theta_j); also stores x_j.  kDctSplit neighbouring
// lanes share node j, lane s summing n = s, s + kDctSplit, ...; the partial sums combine by two
// shuffles in a fixed order.  64 nodes per work-group.
constexpr int kDctSplit = 4;

__global__ void __launch_bounds__(256)
k_dct3(const double* __restrict__ tau, int order, int64_t M, double* __restrict__ w,
       double* __restrict__ x_tab, int damping) {
    static_assert(kDctSplit == 4, "two shuffle steps");
    extern __shared__ double st[];
    // with damping, t(mu~) = sum_n g_n c_n(mu~) tau_n: the factors go onto the moments
    for (int i = threadIdx.x; i <= order; i += 256) st[i] = tau[i] * damping_factor(damping, i, order);
    __syncthreads();
    const int s = threadIdx.x % kDctSplit;
    const int64_t j = ((int64_t)blockIdx.x * 256 + threadIdx.x) / kDctSplit;
    const bool live = j < M;   // no early exit: every lane takes part in the shuffles
    const int64_t mod = 4 * M, q1 = 2 * j + 1, step = (kDctSplit * q1) % mod;
    double acc = 0.0;
    if (live) {
        int64_t q = (s * q1) % mod;   // n q1 mod 4M for n = s
        for (int nn = s; nn <= order; nn += kDctSplit) {
            acc += nn == 0 ? st[0] : 2.0 * st[nn] * node_cos(q, M);
            q += step;
            if (q >= mod) q -= mod;
        }
    }
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    if (live && s == 0) {
        w[j] = acc;
        x_tab[j] = node_cos(q1, M);
    }
}

constexpr int kBisectThreads = 1024;
// Bisection steps per multi-point pass of the single-problem search (seven points side by side,
// two wavefronts each).  Measured search time (DCT-III + search) at N = 256 / 1000 / 2000,
// float64: one step per pass 0.149 / 0.182 / 0.173 ms; two 0.126 / 0.157 / 0.151; three 0.104 /
// 0.137 / 0.131; four 0.109 / 0.142 / 0.134; mu, trace and D bit for bit the same in every case.
constexpr int kBisectLevels = 3;

// mu search of one problem (modes 0 bisection / 1 safeguarded Newton, search_dev.h); scratch:
// M doubles for the tail sums
__global__ void __launch_bounds__(kBisectThreads)
k_bisect(const double* __restrict__ w, const double* __restrict__ x, int64_t M, DevScalars* s, int mode,
         double* __restrict__ scratch) {
    constexpr int NP = (1 << kBisectLevels) - 1;
    __shared__ double smem[kBisectThreads / 64];
    __shared__ double part[kBisectThreads / 64];
    __shared__ double win[4 * NP];
    __shared__ double tout[NP];
    mu_search_one<kBisectThreads, kBisectLevels>(M, w, x, *s, mode, 0.0, 0.0, smem, scratch, part, win, tout);
}

}  // namespace

hipError_t launch_set_scalars(DevScalars* s, double emin, double emax, double beta, double mu,
                              int has_mu, double n_elec, double tol, int max_iter, hipStream_t st,
                              int bounds_on_device) {
    hipLaunchKernelGGL(k_set_scalars, dim3(1), dim3(1), 0, st, s, emin, emax, beta, mu, has_mu,
                       n_elec, tol, max_iter, bounds_on_device);
    return hipGetLastError();
}

hipError_t launch_fermi_coeffs(int order, int M, const DevScalars* s, double* f_tab, double* c_out,
                               hipStream_t st, int damping) {
    hipLaunchKernelGGL(k_fermi_table, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st,
                       (int64_t)M, s, f_tab);
    hipLaunchKernelGGL(k_dct2, dim3((unsigned)(order + 1)), dim3(256), 0, st, (int64_t)M,
                       (const double*)f_tab, c_out, order, damping);
    return hipGetLastError();
}

// Two Clenshaw chains for the giant steps: with T_{h+j} = 2 T_h T_j - T_{h-j} (eq. "identity"
// with a = h, b = j), sum_{l<m} T_l(Y) R_l = sum_{l<h} T_l(Y) R''_l + T_h(Y) sum_{j<m-h} T_j(Y) R'_j,
// R'_0 = R_h, R'_j = 2 R_{h+j}, R''_{h-j} = R_{h-j} - R_{h+j} (1 <= j < m - h <= h).  Applied to
// the block coefficients in place: block h + j then holds R'_j.
namespace {
__global__ void k_split_blocks(double* __restrict__ coef, int k, int m, int h) {
    const int i = threadIdx.x;
    if (i >= k) return;
    for (int j = 1; h + j < m; ++j) {
        const double up = coef[(h + j) * k + i];
        coef[(h - j) * k + i] -= up;
        coef[(h + j) * k + i] = 2.0 * up;
    }
}
}  // namespace

hipError_t launch_split_blocks(double* coef, int k, int m, int h, hipStream_t st) {
    if (k > kMaxBlocks || m > kMaxBlocks || h < 1 || m - h > h) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_split_blocks, dim3(1), dim3(64), 0, st, coef, k, m, h);
    return hipGetLastError();
}

hipError_t launch_block_coeffs(const double* c, int order, int k, int m, int form, double* coef,
                               hipStream_t st) {
    if (k > kMaxBlocks || m > kMaxBlocks) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_block_coeffs, dim3(1), dim3(64), 0, st, c, order, k, m, form, coef);
    return hipGetLastError();
}

hipError_t launch_assemble_moments(const double* tr_baby, const double* gram, int k, int m,
                                   int order, int64_t n, double* tau, hipStream_t st) {
    hipLaunchKernelGGL(k_assemble_moments, dim3(1), dim3(64), 0, st, tr_baby, gram, k, m, order, n, tau);
    return hipGetLastError();
}

hipError_t launch_dct3(const double* tau, int order, int M, double* w, double* x_tab,
                       hipStream_t st, int damping) {
    const size_t shmem = sizeof(double) * (size_t)(order + 1);
    const int64_t threads = (int64_t)M * kDctSplit;
    hipLaunchKernelGGL(k_dct3, dim3((unsigned)((threads + 255) / 256)), dim3(256), shmem, st, tau, order,
                       (int64_t)M, w, x_tab, damping);
    return hipGetLastError();
}

hipError_t launch_bisect(const double* w, const double* x_tab, int M, DevScalars* s, int mode, double* scratch,
                         hipStream_t st) {
    if (mode < 0 || mode > 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bisect, dim3(1), dim3(kBisectThreads), 0, st, w, x_tab, (int64_t)M, s, mode, scratch);
    return hipGetLastError();
}

}  // namespace chebdm
