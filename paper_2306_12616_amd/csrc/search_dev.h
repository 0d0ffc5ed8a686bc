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
//   mode 2  start guess g (the learned network's): Newton steps from g, each
//           evaluation moving the low or the high end of a bracket to its
//           point, until both ends are points where t was evaluated (then
//           safeguarded Newton inside, as mode 1) or the search converges.
//           If a step is undefined (t' <= 0), leaves [-1, 1] or moves further
//           than delta from g, or no bracket forms within kLearnedSteps
//           evaluations, it falls back to plain bisection between the ends
//           found so far and whichever of -1, 1 is still unchecked.
// ERR_BRACKET unless t(-1) < N_e < t(1) (checked for each end not yet known from
// an evaluated point).
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

// Saturated tails by blocks of kQBlock consecutive nodes.  The nodes x_j = cos(pi (j + 1/2) / M)
// fall with j, so for a given mu~ the nodes split into a head (z > kSat: skipped), a window and a
// tail (z < -kSat: occupation exactly 1).  tail_sums stores in blk[b] the sum of w over blocks
// b..nb-1 (blk[nb] = 0), once per search; a pass then visits only the blocks that meet the window
// (found from arccos of its ends, widened by two nodes) and adds the tail as one suffix sum.  It
// classifies every node as the full pass does, so only the order of the additions changes.
constexpr int kQBlock = 256;

// Evaluations the learned start may spend before it holds a bracket.
constexpr int kLearnedSteps = 8;

// Node count of a trace window above which a multi-point bisection pass (one wavefront per
// point) would be slower than a single point on the whole work-group.
constexpr int64_t kWideWindow = 2048;

// blk: nb + 1 doubles of global scratch, nb = ceil(M / kQBlock).  Deterministic.
template <int NT>
__device__ void tail_sums(const double* __restrict__ w, int64_t M, double* __restrict__ blk) {
    __shared__ double chunk[NT];
    const int64_t nb = (M + kQBlock - 1) / kQBlock;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int64_t b = wid; b < nb; b += NT / 64) {   // one wavefront per block
        double v = 0.0;
#pragma unroll
        for (int u = 0; u < kQBlock / 64; ++u) {
            const int64_t j = b * kQBlock + u * 64 + lane;
            v += j < M ? w[j] : 0.0;
        }
        v = wave_sum(v);
        if (lane == 0) blk[b] = v;
    }
    __syncthreads();
    // suffix sums: thread i owns blocks [i C, (i + 1) C)
    const int64_t C = (nb + NT - 1) / NT, b0 = threadIdx.x * C, b1 = b0 + C < nb ? b0 + C : nb;
    double own = 0.0;
    for (int64_t b = b0; b < b1; ++b) own += blk[b];
    chunk[threadIdx.x] = own;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = NT - 1; i >= 0; --i) {
            const double v = chunk[i];
            chunk[i] = s;   // sum over the chunks after i
            s += v;
        }
    }
    __syncthreads();
    double s = chunk[threadIdx.x];
    for (int64_t b = b1 - 1; b >= b0; --b) {
        s += blk[b];
        blk[b] = s;
    }
    if (threadIdx.x == 0) blk[nb] = 0.0;
    __syncthreads();
}

// Node range [j0, j1) of the blocks that meet the window of mu~, and the tail sum past it.
__device__ inline void pass_window(double mu_s, double beta_s, int64_t M, const double* __restrict__ blk,
                                   int64_t& j0, int64_t& j1, double& tail) {
    const double a = mu_s - kSat / beta_s, b = mu_s + kSat / beta_s;
    const double per = (double)M / 3.141592653589793;   // nodes per radian of theta
    int64_t jhi = M - 1, jlo = 0;                       // x_j < a for j > jhi, x_j > b for j < jlo
    if (a > -1.0) {
        const double v = floor(acos(a) * per - 0.5) + 2.0;
        if (v < (double)(M - 1)) jhi = v < 0.0 ? 0 : (int64_t)v;
    }
    if (b < 1.0) {
        const double v = ceil(acos(b) * per - 0.5) - 2.0;
        if (v > 0.0) jlo = v > (double)(M - 1) ? M - 1 : (int64_t)v;
    }
    if (jlo > jhi) jlo = jhi;
    const int64_t bl = jlo / kQBlock, bh = jhi / kQBlock;
    j0 = bl * kQBlock;
    j1 = (bh + 1) * kQBlock < M ? (bh + 1) * kQBlock : M;
    tail = blk[bh + 1];
}

// Nodes j = j0 + threadIdx.x + i NT in increasing i, below j1; the loads of U consecutive i are
// issued together (the search is a chain of dependent passes, so load latency is what it waits
// on).  Slots past j1 add w = 0 with an in-range x, which leaves the sum unchanged.  tail is
// added to t once.
template <int NT, bool SLOPE>
__device__ __forceinline__ void trace_pass(double mu_s, const double* __restrict__ w, const double* __restrict__ x,
                                           int64_t M, double beta_s, double* smem, double& t, double& dt,
                                           const double* __restrict__ blk = nullptr) {
    constexpr int U = 4;
    int64_t j0 = 0, j1 = M;
    double tail = 0.0;
    if (blk) pass_window(mu_s, beta_s, M, blk, j0, j1, tail);
    double acc = threadIdx.x == 0 ? tail : 0.0, accd = 0.0;
    for (int64_t j = j0 + threadIdx.x; j < j1; j += (int64_t)U * NT) {
        double xs[U], ws[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t jj = j + (int64_t)u * NT;
            xs[u] = jj < j1 ? x[jj] : 0.0;
            ws[u] = jj < j1 ? w[jj] : 0.0;
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

// t at P points in one pass: point p by the G = NT / (64 P) wavefronts p G .. p G + G - 1 (any
// left over idle); thread (g, lane) of a point's group adds the nodes j0 + 64 g + lane + k 64 G,
// k = 0, 1, ..., in order (loads of U consecutive k issued together), the group's lane 0 of
// wavefront 0 also its saturated tail, and the group's wavefront sums are added in order.  With
// P = 1 that is exactly trace_pass<NT, false>; with more points the passes run side by side
// instead of one after another, which is what the chain of dependent evaluations waits on.
// Thread p < P brings point p in mu_mine.  Shared: win (4 P doubles: each point's node range,
// tail sum and mu~), part (NT / 64 doubles), tout (P doubles, the results, valid on return).
template <int NT, int P>
__device__ __forceinline__ void trace_pass_groups(double mu_mine, const double* __restrict__ w,
                                                  const double* __restrict__ x, int64_t M, double beta_s,
                                                  double* part, double* win, double* tout,
                                                  const double* __restrict__ blk) {
    constexpr int U = 4, NW = NT / 64, G = NW / P;
    static_assert(G >= 1, "at least one wavefront per point");
    if (threadIdx.x < P) {
        int64_t j0 = 0, j1 = M;
        double tail = 0.0;
        if (blk) pass_window(mu_mine, beta_s, M, blk, j0, j1, tail);
        win[4 * threadIdx.x] = (double)j0;
        win[4 * threadIdx.x + 1] = (double)j1;
        win[4 * threadIdx.x + 2] = tail;
        win[4 * threadIdx.x + 3] = mu_mine;
    }
    __syncthreads();
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int p = wid / G, g = wid % G;
    double a = 0.0;
    if (p < P) {
        const int64_t j0 = (int64_t)win[4 * p], j1 = (int64_t)win[4 * p + 1];
        const double mu_s = win[4 * p + 3];
        constexpr int64_t S = 64 * G;
        if (g == 0 && lane == 0) a = win[4 * p + 2];
        for (int64_t j = j0 + 64 * g + lane; j < j1; j += U * S) {
            double xs[U], ws[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t jj = j + u * S;
                xs[u] = jj < j1 ? x[jj] : 0.0;
                ws[u] = jj < j1 ? w[jj] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const double z = beta_s * (xs[u] - mu_s);
                if (z < -kSat) {
                    a += ws[u];
                } else if (z <= kSat) {
                    const double f = 1.0 / (1.0 + exp(z));
                    a += f * ws[u];
                }
            }
        }
    }
    a = wave_sum(a);
    if (lane == 0) part[wid] = a;
    __syncthreads();
    if (threadIdx.x < P) {
        double r = 0.0;
#pragma unroll
        for (int gg = 0; gg < G; ++gg) r += part[threadIdx.x * G + gg];
        tout[threadIdx.x] = r / (double)M;
    }
    __syncthreads();
}

// Bisection LV steps per pass: the 2^LV - 1 midpoints that the next LV steps can visit (the
// same 0.5 (lo + hi) of the same ends: node q of the heap-ordered tree is reached by halving
// [lo, hi] along the path of q's index, children 2q + 1 for t >= N_e, the left half, and
// 2q + 2) are evaluated side by side (trace_pass_groups), then the steps are taken from those
// values with the stopping rule checked after each, so the sequence of brackets, the step count
// and the stopping point are those of one-at-a-time bisection on the same trace values.  A pass
// whose first window holds more than kWideWindow nodes (small beta', or a coarse bracket near
// the ends) takes one step on all wavefronts instead.  Shared: part, win, tout as for
// trace_pass_groups with P = 2^LV - 1.
template <int NT, int LV>
__device__ void bisect_levels(int64_t M, const double* __restrict__ w, const double* __restrict__ x, double beta_s,
                              double ne, double tol, int max_iter, double* part, double* win, double* tout,
                              const double* __restrict__ blk, double& lo, double& hi, double& mid, double& t_mid,
                              int& iters, int& status) {
    constexpr int NP = (1 << LV) - 1;
    int it = 1;
    bool stop = max_iter < 1;
    while (!stop) {
        const double root = 0.5 * (lo + hi);
        int64_t j0 = 0, j1 = M;
        double tail;
        if (blk) pass_window(root, beta_s, M, blk, j0, j1, tail);
        int levels = LV;
        if (j1 - j0 > kWideWindow) {
            trace_pass_groups<NT, 1>(root, w, x, M, beta_s, part, win, tout, blk);
            levels = 1;
        } else {
            double mine = root;
            if (threadIdx.x < NP) {   // walk down to node threadIdx.x
                const int q1 = (int)threadIdx.x + 1;
                const int depth = 31 - __clz(q1);
                double l = lo, h = hi;
                for (int b = depth - 1; b >= 0; --b) {
                    const double m = 0.5 * (l + h);
                    if ((q1 >> b) & 1) l = m;   // right child: [m, h]
                    else h = m;
                }
                mine = 0.5 * (l + h);
            }
            trace_pass_groups<NT, NP>(mine, w, x, M, beta_s, part, win, tout, blk);
        }
        int k = 0;
        for (int lev = 0; lev < levels; ++lev) {
            mid = win[4 * k + 3];
            t_mid = tout[k];
            iters = it;
            if (fabs(t_mid - ne) < tol) {
                status = CHEBDM_OK;
                stop = true;
                break;
            }
            const bool below = t_mid < ne;
            if (below) lo = mid;
            else hi = mid;
            if (hi - lo < 4.0 * ulp_spacing(mid) || ++it > max_iter) {
                stop = true;
                break;
            }
            k = 2 * k + (below ? 2 : 1);
        }
        __syncthreads();   // win and tout are rewritten by the next pass
    }
}

// Writes mu_s, trace, iters, evals, learned, status, lo, hi of d (thread 0).  scratch: nullptr,
// or M doubles of global memory for the tail sums (used from M >= 4 kQBlock on).  LV > 0 (with
// shared part of NT / 64 doubles, win of 4 (2^LV - 1) and tout of 2^LV - 1): the bisection of
// mode 0 takes up to LV steps per pass (bisect_levels) and the bracket check evaluates both ends
// side by side.
template <int NT, int LV = 0>
__device__ void mu_search_one(int64_t M, const double* __restrict__ w, const double* __restrict__ x, DevScalars& d,
                              int mode, double guess, double delta, double* smem, double* scratch = nullptr,
                              double* part = nullptr, double* win = nullptr, double* tout = nullptr) {
    const double* blk = nullptr;
    if (scratch && M >= 4 * kQBlock) {
        tail_sums<NT>(w, M, scratch);
        blk = scratch;
    }
    const double beta_s = d.beta_s, ne = d.n_elec, tol = d.tol;
    const int max_iter = d.max_iter;
    int evals = 0, learned = 0, iters = 0, status = CHEBDM_WARN_NOCONV;
    double lo = -1.0, hi = 1.0, mu0 = 0.0, t_lo, t_hi, unused;
    bool have_lo = false, have_hi = false;   // an end is a point where t was evaluated
    double mid = 0.0, t_mid = NAN;
    bool done = false;
    if (mode == 2) {
        const double g = fmin(fmax(isfinite(guess) ? guess : 0.0, -1.0), 1.0);
        mid = g;
        for (int it = 1; it <= kLearnedSteps && it <= max_iter; ++it) {
            double dt;
            trace_pass<NT, true>(mid, w, x, M, beta_s, smem, t_mid, dt, blk);
            ++evals;
            if (fabs(t_mid - ne) < tol) {
                status = CHEBDM_OK;
                learned = 1;
                done = true;
                break;
            }
            if (t_mid < ne) {
                lo = mid;
                have_lo = true;
            } else {
                hi = mid;
                have_hi = true;
            }
            if (have_lo && have_hi) {   // bracketed: safeguarded Newton inside from here
                learned = 1;
                double cand = mid - (t_mid - ne) / dt;
                if (!(dt > 0.0) || !(cand > lo && cand < hi)) cand = 0.5 * (lo + hi);
                if (hi - lo < 4.0 * ulp_spacing(mid)) {
                    done = true;
                    break;
                }
                mu0 = cand;
                break;
            }
            const double cand = mid - (t_mid - ne) / dt;
            if (!(dt > 0.0) || !(cand > -1.0 && cand < 1.0) || !(fabs(cand - g) <= delta)) break;
            mid = cand;
        }
    }
    if constexpr (LV > 0) {
        if (!done && !learned && !have_lo && !have_hi) {
            trace_pass_groups<NT, 2>(threadIdx.x == 0 ? -1.0 : 1.0, w, x, M, beta_s, part, win, tout, blk);
            evals += 2;
            lo = -1.0;
            hi = 1.0;
            t_lo = tout[0];
            t_hi = tout[1];
            have_lo = have_hi = true;   // both ends checked here; the block below only tests them
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
    }
    if (!done && !learned) {
        // the ends not known from an evaluated point are -1 and 1, checked here
        if (!have_lo) {
            lo = -1.0;
            trace_pass<NT, false>(lo, w, x, M, beta_s, smem, t_lo, unused, blk);
            ++evals;
        } else {
            t_lo = -INFINITY;
        }
        if (!have_hi) {
            hi = 1.0;
            trace_pass<NT, false>(hi, w, x, M, beta_s, smem, t_hi, unused, blk);
            ++evals;
        } else {
            t_hi = INFINITY;
        }
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
    if (done) {
        // converged (or collapsed) in the learned start
    } else if (LV > 0 && mode == 0) {
        if constexpr (LV > 0)
            bisect_levels<NT, LV>(M, w, x, beta_s, ne, tol, max_iter, part, win, tout, blk, lo, hi, mid, t_mid,
                                  iters, status);
    } else if (mode == 0 || (mode == 2 && !learned)) {
        for (int it = 1; it <= max_iter; ++it) {
            mid = 0.5 * (lo + hi);
            trace_pass<NT, false>(mid, w, x, M, beta_s, smem, t_mid, unused, blk);
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
            trace_pass<NT, true>(mid, w, x, M, beta_s, smem, t_mid, dt, blk);
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
