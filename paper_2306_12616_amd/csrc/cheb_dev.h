// Scalar device helpers of the coefficient, moment and bisection kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace chebdm {

// cos(pi q / (2M)) for the Chebyshev-Gauss angles theta_j = pi (j + 1/2) / M:
// q / (2M) is exact because 2M is a power of two, so every cosine is a
// correctly reduced cospi (q = n (2j+1) mod 4M is formed in integers).
__device__ inline double node_cos(int64_t q, int64_t M) { return cospi((double)q / (double)(2 * M)); }

// 1 / (1 + exp(beta'(x - mu~)))  (eq. "fermifunc" in scaled variables)
__device__ inline double fermi_scaled(double x, double beta_s, double mu_s) {
    return 1.0 / (1.0 + exp(beta_s * (x - mu_s)));
}

// Jackson damping factor g_n of a series of N = order + 1 terms (kernel polynomial method):
// g_n = [(N - n + 1) cos(pi n/(N+1)) + sin(pi n/(N+1)) cot(pi/(N+1))] / (N + 1); 1 if damping == 0.
__device__ inline double damping_factor(int damping, int n, int order) {
    if (damping == 0) return 1.0;
    const double N1 = (double)order + 2.0;   // N + 1
    const double u = (double)n / N1;
    return (((double)order + 2.0 - n) * cospi(u) + sinpi(u) * cospi(1.0 / N1) / sinpi(1.0 / N1)) / N1;
}

// Distance from |v| to the next larger double (|v| = 0 is taken as 1e-300).
__device__ inline double ulp_spacing(double v) {
    const double a = v != 0.0 ? fabs(v) : 1e-300;
    return nextafter(a, INFINITY) - a;
}

// Quadrature size M = 2^ceil(log2 max(2(L+1), L/2 + 7 beta' + 64)); -1 if above 2^29.
__host__ __device__ inline int64_t quad_rule(int order, double beta_s) {
    const double need = fmax(2.0 * (order + 1), 0.5 * order + 7.0 * beta_s + 64.0);
    int64_t m = 1;
    int lg = 0;
    while ((double)m < need) {
        m <<= 1;
        if (++lg > 29) return -1;
    }
    return m;
}

}  // namespace chebdm
