// Chemical-potential search on the quadrature trace (device code shared by
// the single-problem and the batched kernels; one work-group per problem).
//
// With w_j the DCT-III of the trace moments and x_j the Chebyshev-Gauss
// nodes, the electron count at scaled chemical potential mu~ is
//     t(mu~) = (1/M) sum_j f(x_j; mu~) w_j = sum_n c_n(mu~) tau_n,
// and its derivative t'(mu~) = (1/M) sum_j beta' f (1 - f) w_j comes from the
// same pass.  Every mode stops at |t - N_e| < tol, at a bracket narrower
// than 4 ulp of the iterate (WARN_NOCONV), or after max_iter steps.
//   mode 0  bisection on [-1, 1] (midpoint rule)
//   mode 1  safeguarded Newton on [-1, 1] from mu~ = 0: every evaluation
//           shrinks the bracket, and a Newton step that leaves it becomes a
//           bisection step
//   mode 2  start guess g (the learned network's): if t(g - delta) < N_e <
//           t(g + delta), safeguarded Newton from g inside that bracket;
//           otherwise plain bisection on [-1, 1] (the fallback)
// ERR_BRACKET unless t(-1) < N_e < t(1) (checked whenever [-1, 1] is used).
#pragma once

#include "cheb_dev.h"
#include "internal.h"
#include "reduce.h"

namespace chebdm {
namespace {

// Occupations saturate away from mu~: for z = beta'(x - mu~) below -kSat, 1/(1 + e^z) is 1
// in double precision (e^-50 is far below half an ulp of 1), and above kSat it is below
// 2e-22, so it is taken as 0; with |w_j| <= 2 sum_n |tau_n| that changes t by < 1e-15 of n.
// The nodes are ordered in x, so whole wavefronts skip the exponential except near mu~.
constexpr double kSat = 50.0;

// Nodes j = threadIdx.x + i NT in increasing i; the loads of U consecutive i are issued
// together (the search is a chain of dependent passes, so load latency is what it waits on).
// Slots past M add w = 0 with an in-range x, which leaves the sum unchanged.
template <int NT, bool SLOPE>
__device__ __forceinline__ void trace_pass(double mu_s, const double* __restrict__ w, const double* __restrict__ x,
                                           int64_t M, double beta_s, double* smem, double& t, double& dt) {
    constexpr int U = 4;
    double acc = 0.0, accd = 0.0;
    for (int64_t j = threadIdx.x; j < M; j += (int64_t)U * NT) {
        double xs[U], ws[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t jj = j + (int64_t)u * NT;
            xs[u] = jj < M ? x[jj] : 0.0;
            ws[u] = jj < M ? w[jj] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double z = beta_s * (xs[u] - mu_s);
            if (z < -kSat) {
                acc += ws[u];
            } else if (z <= kSat) {
                const double f = 1.0 / (1.0 + exp(z));
                acc += f * ws[u];
                if (SLOPE) accd += beta_s * f * (1.0 - f) * ws[u];
            }
        }
    }
    t = block_sum<NT>(acc, smem) / (double)M;
    dt = SLOPE ? block_sum<NT>(accd, smem) / (double)M : 0.0;
}

// Writes mu_s, trace, iters, evals, learned, status, lo, hi of d (thread 0).
template <int NT>
__device__ void mu_search_one(int64_t M, const double* __restrict__ w, const double* __restrict__ x, DevScalars& d,
                              int mode, double guess, double delta, double* smem) {
    const double beta_s = d.beta_s, ne = d.n_elec, tol = d.tol;
    const int max_iter = d.max_iter;
    int evals = 0, learned = 0, iters = 0, status = CHEBDM_WARN_NOCONV;
    double lo = -1.0, hi = 1.0, mu0 = 0.0, t_lo, t_hi, unused;
    bool bracketed = false;
    if (mode == 2) {
        double g = isfinite(guess) ? guess : 0.0;
        g = fmin(fmax(g, -1.0), 1.0);
        lo = fmax(-1.0, g - delta);
        hi = fmin(1.0, g + delta);
        trace_pass<NT, false>(lo, w, x, M, beta_s, smem, t_lo, unused);
        trace_pass<NT, false>(hi, w, x, M, beta_s, smem, t_hi, unused);
        evals += 2;
        if (t_lo < ne && ne < t_hi) {
            bracketed = true;
            learned = 1;
            mu0 = g;
        }
    }
    double mid = 0.0, t_mid = NAN;
    if (!bracketed) {
        lo = -1.0;
        hi = 1.0;
        trace_pass<NT, false>(lo, w, x, M, beta_s, smem, t_lo, unused);
        trace_pass<NT, false>(hi, w, x, M, beta_s, smem, t_hi, unused);
        evals += 2;
        if (!(t_lo < ne && ne < t_hi)) {
            if (threadIdx.x == 0) {
                d.mu_s = NAN;
                d.trace = NAN;
                d.iters = 0;
                d.evals = evals;
                d.learned = 0;
                d.status = CHEBDM_ERR_BRACKET;
                d.lo = lo;
                d.hi = hi;
            }
            return;
        }
    }
    if (mode == 0 || (mode == 2 && !learned)) {
        for (int it = 1; it <= max_iter; ++it) {
            mid = 0.5 * (lo + hi);
            trace_pass<NT, false>(mid, w, x, M, beta_s, smem, t_mid, unused);
            iters = it;
            if (fabs(t_mid - ne) < tol) {
                status = CHEBDM_OK;
                break;
            }
            if (t_mid < ne) lo = mid;
            else hi = mid;
            if (hi - lo < 4.0 * ulp_spacing(mid)) break;
        }
    } else {
        mid = mu0;
        for (int it = 1; it <= max_iter; ++it) {
            double dt;
            trace_pass<NT, true>(mid, w, x, M, beta_s, smem, t_mid, dt);
            iters = it;
            if (fabs(t_mid - ne) < tol) {
                status = CHEBDM_OK;
                break;
            }
            if (t_mid < ne) lo = mid;
            else hi = mid;
            double cand = mid - (t_mid - ne) / dt;
            if (!(dt > 0.0) || !(cand > lo && cand < hi)) cand = 0.5 * (lo + hi);
            if (hi - lo < 4.0 * ulp_spacing(mid)) break;
            mid = cand;
        }
    }
    evals += iters;
    if (threadIdx.x == 0) {
        d.mu_s = mid;
        d.trace = t_mid;
        d.iters = iters;
        d.evals = evals;
        d.learned = learned;
        d.status = status;
        d.lo = lo;
        d.hi = hi;
    }
}

}  // namespace
}  // namespace chebdm
