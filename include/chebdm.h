/*
 * chebdm.h - C ABI of the dense Chebyshev Fermi-operator library for MI355X (gfx950).
 *
 * The library builds the single-particle density matrix
 *     D = f(H) = [I + exp(beta (H - mu I))]^{-1}                (paper, Sec. II.B, eq. "fermi")
 * of a dense symmetric Hamiltonian without diagonalisation, as the degree-L
 * Chebyshev expansion D_L = sum_{n<=L} c_n T_n(H~) evaluated with the
 * O(sqrt(L)) baby-step/giant-step scheme of Sec. II.B (eqs. "ansatz",
 * "ansatz3"): k-1 products for T_2..T_k, m-1 products over T_k blocks, L = km-1.
 * All device work runs in the library's own HIP kernels.
 *
 * Conventions shared by every entry point
 *   - Matrices are dense, float64, row-major with a leading dimension
 *     ld >= n (element (i,j) at p[i*ld + j]).  H must be symmetric; it is not
 *     checked.  Because H and D are symmetric, row- and column-major agree.
 *   - Pointers named d* are device pointers on the handle's device and stay
 *     owned by the caller; pointers named h* / *_out are host pointers.
 *   - Work is ordered on the handle's HIP stream.  Entry points that return
 *     host values (bounds, coefficients, mu, info, moments) synchronise that
 *     stream before returning; chebdm_density with info == NULL does not.
 *   - dD must not alias dH.  The library owns a workspace of about
 *     (k + m) * ld^2 elements, grown on demand and kept until chebdm_destroy.
 *   - emin/emax arguments: pass NAN (both) to let the call compute bounds of H
 *     itself (Gershgorin's, or Lanczos' with opts->bounds), or the caller's own
 *     outer bounds of the spectrum.
 *   - Return value: CHEBDM_OK (0), a positive warning (result usable), or a
 *     negative error; chebdm_last_error() then describes the failure
 *     (thread-local string).  No C++ exception crosses this interface.
 *   - A handle must not be used from two threads at once.
 *   - chebdm_density and chebdm_mu_search capture their device work (after
 *     the bounds) into a HIP graph on a stream of the handle's own and replay
 *     it on the handle's stream while the call's arguments are unchanged
 *     (pointers, sizes, beta, mu or n_elec, options, quadrature size and
 *     workspace; new contents under the same pointers are fine).  The handle
 *     keeps one graph per kind of call (mu search with and without D,
 *     density).  With launch timing on (chebdm_profile_enable) they run
 *     eagerly.  Neither may be called while the handle's stream is itself
 *     being captured (they synchronise it).
 */
#ifndef CHEBDM_H
#define CHEBDM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CHEBDM_ABI_VERSION 4

typedef struct chebdm_ctx* chebdm_handle;

/* Arithmetic of the matrix products (the bounds, coefficients, traces,
 * moments and the mu search are always float64). */
enum chebdm_prec {
    CHEBDM_FP64 = 0,   /* float64 MFMA products, float64 matrices            */
    CHEBDM_FP32 = 1,   /* float32 MFMA products, float32 matrices            */
    CHEBDM_BF16X3 = 2, /* float32 matrices, products as three bfloat16 MFMA  */
                       /* terms hi*hi + hi*lo + lo*hi, float32 accumulation  */
                       /* (x = hi + lo; about 2^-16 relative per product)    */
    CHEBDM_BF16X6 = 3  /* float32 matrices, x = hi + mid + lo in bfloat16,   */
                       /* six MFMA terms down to 2^-16 (hh hm mh hl lh mm),  */
                       /* float32 accumulation: about float32 accuracy       */
};

/* Order of the baby-step products T_2..T_k and of the mu search's ladder T_2k, T_3k, ...
   (both orders give the same matrices up to rounding). */
enum chebdm_baby {
    CHEBDM_BABY_AUTO = 0,       /* baby steps: stages for CHEBDM_FP64, odd chains for     */
                                /* CHEBDM_FP32, sequential for the split-bf16 precisions; */
                                /* ladder: stages for CHEBDM_FP64 and CHEBDM_FP32,        */
                                /* sequential for the split-bf16 precisions; CHEBDM_FP32  */
                                /* with k > 24 (order >= 576): sequential for both        */
    CHEBDM_BABY_STAGES = 1,     /* Algorithm 1: ceil(log2 k) stages of independent        */
                                /* products T_{i+u} = 2 T_i T_u - T_{i-u}, one launch each */
    CHEBDM_BABY_SEQUENTIAL = 2, /* T_{i+1} = 2 T_1 T_i - T_{i-1}: errors grow ~i instead  */
                                /* of ~i^2, which matters for float32 / bf16 products     */
    CHEBDM_BABY_ODD_CHAINS = 3  /* T_2..T_s (the same way with a smaller step, or one by  */
                                /* one), then s interleaved chains                       */
                                /* T_{i+s} = 2 T_s T_i - T_{|i-s|}, one launch of s       */
                                /* products per round; s odd >= 3, chosen for the fewest  */
                                /* launches (5 for k = 23).  T_s of odd s is as small as  */
                                /* T_1 where the spectrum sits well inside the bounds, so */
                                /* the errors stay those of the sequential order          */
};

/* How the giant steps combine the blocks (all give the same polynomial). */
enum chebdm_giant {
    CHEBDM_GIANT_COMPOSITION = 0, /* sum_l T_l(T_k) R_l by Clenshaw over l (default);  */
                                  /* the library picks one, two or four chains (below; */
                                  /* four while a product has < 1024 64-tiles)        */
    CHEBDM_GIANT_POWER = 1,       /* paper's sum_j T_k^j S_j by Horner (eq. "ansatz") */
    CHEBDM_GIANT_ONE_CHAIN = 2,   /* composition form, one Clenshaw chain: m-1 steps  */
    CHEBDM_GIANT_TWO_CHAINS = 3,  /* composition form as two chains of about m/2      */
                                  /* steps run side by side, joined by one product    */
                                  /* with T_h(T_k), h = ceil(m/2) (via eq. "identity"),*/
                                  /* when that matrix comes from the moment ladder:   */
                                  /* chebdm_mu_search with D and m >= 4; otherwise one */
                                  /* chain.  Same m-1 products, half the sequential   */
                                  /* launches, two products per launch.               */
    CHEBDM_GIANT_FOUR_CHAINS = 4  /* both halves of the two chains split again at     */
                                  /* q = ceil(h/2) the same way: four chains of about */
                                  /* m/4 steps side by side, then one launch of two   */
                                  /* products with T_q(T_k), then the product with    */
                                  /* T_h(T_k).  Needs m >= 8 and the ladder as above; */
                                  /* otherwise as CHEBDM_GIANT_TWO_CHAINS.  Same m-1  */
                                  /* products in about m/4 + 2 launches.              */
};

/* How chebdm_mu_search finds mu~ on the quadrature trace t(mu~) (both stop
 * at |t - N_e| < tol, at a bracket under 4 ulp, or after max_iter steps). */
enum chebdm_search {
    CHEBDM_SEARCH_BISECTION = 0, /* midpoint rule on [-1, 1]                          */
    CHEBDM_SEARCH_NEWTON = 1     /* safeguarded Newton from 0 with t' from the same   */
                                 /* quadrature; a step leaving the bracket bisects   */
};

/* Optional damping of the expansion (not in the paper, which truncates plainly
 * and notes the Gibbs oscillations): c_n -> g_n c_n in the density and in the
 * trace t(mu~) the search solves, g_n the Jackson factors of the kernel
 * polynomial method for N = L + 1 terms,
 *   g_n = [(N-n+1) cos(pi n/(N+1)) + sin(pi n/(N+1)) cot(pi/(N+1))] / (N+1).
 * The damped polynomial of a function in [0, 1] stays in [0, 1]. */
enum chebdm_damping {
    CHEBDM_DAMPING_NONE = 0,
    CHEBDM_DAMPING_JACKSON = 1
};

/* Where NaN bounds are resolved from (the paper needs the extreme eigenvalues
 * e_a, e_b, Sec. II.B, and names no method).  A tighter interval lowers
 * beta' = beta (emax - emin)/2 and so the truncation error at a given order. */
enum chebdm_bounds_method {
    CHEBDM_BOUNDS_GERSHGORIN = 0, /* Gershgorin discs (always hold the spectrum)       */
    CHEBDM_BOUNDS_LANCZOS = 1     /* chebdm_bounds_lanczos with seed 0: a few Lanczos  */
                                  /* steps, residual-widened, inside Gershgorin's      */
};

enum chebdm_status {
    CHEBDM_OK = 0,
    CHEBDM_WARN_NOCONV = 1,       /* mu search stopped before |t - N_e| < tol    */
    CHEBDM_ERR_ARG = -1,          /* invalid argument                            */
    CHEBDM_ERR_HIP = -2,          /* a HIP runtime call failed                   */
    CHEBDM_ERR_OOM = -3,          /* workspace allocation failed                 */
    CHEBDM_ERR_NONFINITE = -4,    /* H holds NaN or Inf                          */
    CHEBDM_ERR_BRACKET = -5,      /* N_e not inside (t(mu~=-1), t(mu~=1))        */
    CHEBDM_ERR_UNSUPPORTED = -6   /* option combination not built                */
};

typedef struct {
    int32_t prec;        /* enum chebdm_prec, default CHEBDM_FP64                  */
    int32_t giant_form;  /* enum chebdm_giant, default CHEBDM_GIANT_COMPOSITION    */
    int32_t k_override;  /* baby-step count k; 0 = ceil(sqrt(L+1))                 */
    int32_t n_quad;      /* quadrature nodes M for c_n; 0 = automatic rule         */
    int32_t max_iter;    /* cap on search steps (trace evaluations); 0 = 200       */
    int32_t baby_steps;  /* enum chebdm_baby, default CHEBDM_BABY_AUTO                */
    int32_t search;      /* enum chebdm_search of chebdm_mu_search, default BISECTION */
    int32_t damping;     /* enum chebdm_damping, default CHEBDM_DAMPING_NONE        */
    double tol;          /* target |tr D - N_e| of the mu search; 0 = 1e-10        */
    int32_t bounds;      /* enum chebdm_bounds_method for NaN bounds, default GERSHGORIN */
    int32_t lanczos_steps; /* Lanczos steps; 0 = 40, at most 128                   */
    double bounds_margin;  /* relative widening of the Lanczos bounds; 0 = 0.01    */
} chebdm_opts;

typedef struct {
    int32_t k, m;        /* baby-step count and block count, L + 1 <= k*m           */
    int32_t n_gemm;      /* matrix products executed                               */
    int32_t n_quad;      /* quadrature nodes M used for the coefficients           */
    int32_t iters;       /* search steps after the bracket check (mu search)       */
    int32_t status;      /* same as the return value                               */
    double emin, emax;   /* spectral bounds used                                   */
    double mu;           /* chemical potential used (energy units)                 */
    double trace;        /* tr D in float64 (or t(mu) when no D was built)         */
    double trace_err;    /* |t(mu) - N_e| of the search (mu search only)           */
} chebdm_info;

/* Fill *o with the defaults listed above. */
void chebdm_default_opts(chebdm_opts* o);

/* Version of this ABI (CHEBDM_ABI_VERSION). */
int chebdm_abi_version(void);

/* Thread-local description of the last failure in this thread ("" if none). */
const char* chebdm_last_error(void);

/* Create a handle bound to HIP device `device` and stream `stream`
 * (a hipStream_t; NULL = the legacy default stream).  *out receives the handle. */
int chebdm_create(chebdm_handle* out, int device, void* stream);

/* Release the handle and its workspace (waits for its stream first). */
int chebdm_destroy(chebdm_handle h);

/* Re-bind the handle to another stream on the same device. */
int chebdm_set_stream(chebdm_handle h, void* stream);

/*
 * Spectral bounds of H by Gershgorin's discs (reading of Sec. II.B, which
 * asks for the lowest and highest eigenvalues e_a, e_b without a method):
 *     emin = min_i (H_ii - r_i),  emax = max_i (H_ii + r_i),  r_i = sum_{j!=i} |H_ij|,
 * summed in float64 in a fixed order (deterministic).
 * dH: n x n, leading dimension ldh >= n.  Writes host doubles *emin, *emax.
 * Errors: CHEBDM_ERR_ARG (n < 1, ldh < n, NULL pointers),
 *         CHEBDM_ERR_NONFINITE (H holds NaN/Inf).
 */
int chebdm_bounds(chebdm_handle h, const double* dH, int64_t n, int64_t ldh,
                  double* emin, double* emax);

/*
 * chebdm_bounds for callers that cannot allocate device memory (code under
 * HIP stream capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same Gershgorin kernels and fold order, with their partial sums in a
 * fixed static device array of 8 MiB (each GPU the library runs on holds one
 * until the process ends; its address is looked up when a handle on that
 * device is created).  The call allocates nothing, does not synchronise and
 * is stream-ordered on the handle's stream.
 * dH: n x n, leading dimension ldh >= n, 1 <= n <= 65535 (larger n:
 * CHEBDM_ERR_ARG).  d_out: device pointer to 2 doubles, receives emin, emax
 * (both NaN when H holds NaN or Inf; there is no read-back to report it).
 * All calls on one device share that device's array: calls that overlap on
 * one device (two streams, two threads) race and must be serialised by the
 * caller.  Errors: CHEBDM_ERR_ARG, CHEBDM_ERR_HIP.
 */
int chebdm_bounds_noalloc(chebdm_handle h, const double* dH, int64_t n, int64_t ldh, double* d_out);

/*
 * Spectral bounds of H from `steps` Lanczos steps (not in the paper; a
 * tighter alternative to Gershgorin's discs for e_a, e_b of Sec. II.B).
 * Start vector: the SplitMix64 generator (Steele, Lea, Flood 2014) of `seed`,
 * output i mapped to 2 (top 53 bits) 2^-53 - 1, normalised.  Step j:
 *     w = H v_j,  alpha_j = v_j.w,  w -= alpha_j v_j + beta_{j-1} v_{j-1},
 *     w -= sum_{i<=j} (v_i.w) v_i (one full reorthogonalisation),
 *     beta_j = ||w||,  v_{j+1} = w / beta_j,
 * all in float64 on the device; it stops early when beta_j <= 1e-12 *
 * max(|g_lo|, |g_hi|), [g_lo, g_hi] the Gershgorin bounds.  With theta the
 * extreme eigenvalues of the k x k tridiagonal (alpha, beta) and
 * r = beta_{k-1}, the result is [theta_min - r, theta_max + r] widened by
 * margin * width on each side and intersected with [g_lo, g_hi] (that
 * interval alone if the intersection is empty).  Once the extreme Ritz
 * values have settled (about ten steps for dense H; the default is 40) the
 * widening by the last residual norm encloses the spectrum in practice, but
 * it is not a proof, and one or two steps can miss the edges; the Gershgorin
 * intersection keeps the result inside a proven enclosure.
 * steps in [1, 128] (min(steps, n) are taken); margin >= 0.
 * Host outputs: *emin, *emax; alpha_out, beta_out (optional, NULL allowed,
 * `steps` doubles each: the tridiagonal, beta_out[k-1] = r); *steps_done
 * (optional): k.  Errors: CHEBDM_ERR_ARG, CHEBDM_ERR_NONFINITE, CHEBDM_ERR_OOM.
 */
int chebdm_bounds_lanczos(chebdm_handle h, const double* dH, int64_t n, int64_t ldh,
                          int32_t steps, double margin, uint64_t seed, double* emin, double* emax,
                          double* alpha_out, double* beta_out, int32_t* steps_done);

/*
 * Commutator check of a density matrix: *out = max_ij |(H D - D H)_ij|.
 * A function of H commutes with it (D is built from H's eigenvectors in
 * Sec. II.A), so this measures how far D is from any function of H; for a
 * float64 expansion it sits at rounding level (about 1e-13 |H|).  H and D
 * must be symmetric (not checked).  Float64 MFMA products on the device
 * (2 n^3 flops); H and D are copied into two matrices of the handle's
 * workspace (which the next density or mu-search call overwrites).
 * dH, dD: n x n device matrices, leading dimensions ldh, ldd >= n.
 * *out: host double (NaN if H or D holds NaN).
 * Errors: CHEBDM_ERR_ARG, CHEBDM_ERR_OOM, CHEBDM_ERR_HIP.
 */
int chebdm_commutator_norm(chebdm_handle h, const double* dH, int64_t ldh, const double* dD, int64_t ldd,
                           int64_t n, double* out);

/*
 * Chebyshev coefficients c_0..c_L of the Fermi function on [emin, emax]
 * (the expansion sum c_n T_n of Sec. II.B; projection is a reading):
 *     c_n = (2 - delta_{n0})/M * sum_{j<M} f(x_j) cos(n theta_j),
 *     theta_j = pi (j + 1/2)/M,  x_j = cos theta_j,
 *     f(x) = 1/(1 + exp(beta' (x - mu~))),  beta' = beta (emax-emin)/2,
 *     mu~ = (mu - (emin+emax)/2) / ((emax-emin)/2)       (eq. "fermifunc").
 * n_quad = M (0 = automatic: 2^ceil(log2 max(2(L+1), L/2 + 7 beta' + 64))).
 * Computed on the device in float64; c_out: host array of order+1 doubles.
 * Errors: CHEBDM_ERR_ARG (order < 0, beta <= 0, emax <= emin, M < L+1).
 */
int chebdm_coeffs(chebdm_handle h, double beta, double mu, double emin, double emax,
                  int32_t order, int32_t n_quad, double* c_out);

/*
 * Density matrix at a given chemical potential mu (Sec. II.B and III.B):
 * bounds (if NaN) -> T_1 = H~ -> coefficients -> block coefficients
 * (power form d of eq. "X", or composition form) -> baby steps T_2..T_k in
 * the stage order of Algorithm 1 -> block sums -> m-1 giant steps -> D.
 * dD: n x n output, leading dimension ldd >= n (only that n x n part is
 * written).  opts may be NULL (defaults).  info may be NULL.
 * Errors: CHEBDM_ERR_ARG, CHEBDM_ERR_NONFINITE, CHEBDM_ERR_OOM, CHEBDM_ERR_HIP,
 *         CHEBDM_ERR_UNSUPPORTED (BF16X3 with the power form).
 */
int chebdm_density(chebdm_handle h, const double* dH, int64_t n, int64_t ldh,
                   double beta, double mu, int32_t order, const chebdm_opts* opts,
                   double emin, double emax, double* dD, int64_t ldd, chebdm_info* info);

/*
 * Chemical potential with tr D_L(mu) = n_elec, then (if dD != NULL) D at it.
 * The trace moments tau_n = tr T_n(H~), n <= L, come from the baby steps and
 * a ladder T_{2k}, ..., T_{(m-1)k} through 2 T_a T_b = T_{a+b} + T_{|a-b|}
 * (eq. "identity"); t(mu~) = sum_n c_n(mu~) tau_n is searched on
 * mu~ in [-1, 1] by bisection (midpoint rule) or, with opts->search =
 * CHEBDM_SEARCH_NEWTON, by safeguarded Newton; both stop when
 * |t - n_elec| < tol, when the bracket is narrower than 4 ulp, or after
 * max_iter steps.
 * Writes *mu_out (energy units, host).  0 < n_elec < n required.
 * Returns CHEBDM_WARN_NOCONV if the bracket collapsed before tol was met.
 * Errors: as chebdm_density, plus CHEBDM_ERR_BRACKET.
 */
int chebdm_mu_search(chebdm_handle h, const double* dH, int64_t n, int64_t ldh,
                     double beta, double n_elec, int32_t order, const chebdm_opts* opts,
                     double emin, double emax, double* mu_out, double* dD, int64_t ldd,
                     chebdm_info* info);

/*
 * Device memory a call of chebdm_density / chebdm_mu_search / chebdm_moments
 * with these sizes and options makes the handle hold (it keeps the largest it
 * has needed): the matrix workspace, (k + m) ld^2 elements (k + m + 1 for
 * the composition form with m >= 4: the two-chain giant steps keep T_h(T_k);
 * k + m + 2 where the giant steps go in four chains: they also keep T_q(T_k))
 * with ld = round_up(n, 128) and 8 (float64) or 4 bytes per element, plus the
 * small buffers sized for opts->n_quad quadrature nodes (2^16 when 0), plus
 * 64 MB of product scratch (partial sums of K-sliced product tiles).
 * Needs no device; h may be NULL.  ERR_ARG on bad sizes or options.
 */
int chebdm_workspace_size(chebdm_handle h, int64_t n, int32_t order, const chebdm_opts* opts,
                          size_t* bytes);

/*
 * Trace moments tau_0..tau_L of T_n(H~) (the quantities the mu search
 * bisects on), computed as in chebdm_mu_search.  tau_out: host, order+1 doubles.
 */
int chebdm_moments(chebdm_handle h, const double* dH, int64_t n, int64_t ldh,
                   int32_t order, const chebdm_opts* opts, double emin, double emax,
                   double* tau_out);

/*
 * Block coefficients for given c_0..c_L (host in, host out), k = opts->k_override
 * or ceil(sqrt(L+1)), m = ceil((L+1)/k).  coef_out: m x k row-major, entry
 * (l, i) is the weight of T_i in block l:
 *   CHEBDM_GIANT_POWER:       d_{i,l} of eq. "ansatz3", from c = X d (eq. "X")
 *                             by back substitution over the row blocks l = m-1..0;
 *   CHEBDM_GIANT_COMPOSITION: e_{l,i} with sum_n c_n T_n = sum_l T_l(T_k) R_l,
 *                             R_l = sum_i e_{l,i} T_i, from the same identity.
 * Runs on the device.  Writes *k_out, *m_out.  coef_out must hold k*m doubles
 * (pass k_out/m_out first with coef_out == NULL to query the size).
 */
int chebdm_block_coeffs(chebdm_handle h, const double* c, int32_t order, int32_t giant_form,
                        int32_t k_override, int32_t* k_out, int32_t* m_out, double* coef_out);

/*
 * Batched form: many Hamiltonians of different n with one common order, run
 * as one HIP graph (captured on the first chebdm_batch_mu_search, replayed
 * afterwards; the caller's pointers, beta and N_e are read from a table
 * uploaded before each replay, so the graph is reused across calls).  Per
 * problem it computes exactly what chebdm_mu_search computes (Gershgorin
 * bounds, or Lanczos bounds inside them with opts->bounds, sequential baby
 * steps, ladder and Gram moments, the mu search, composition-form giant steps
 * in one chain); every product step of all problems is one persistent launch
 * over a list of (problem, tile) items.
 *
 * chebdm_batch_create: count problems of sizes n[p] (1..65535), order >= 2
 *   (k, m >= 2); opts: prec any, giant_form COMPOSITION or ONE_CHAIN, n_quad 0,
 *   search sets the initial search mode (0 or 1, see chebdm_batch_set_search),
 *   bounds / lanczos_steps / bounds_margin as for one problem (the Lanczos
 *   workspace is count x lanczos_work(max n) doubles, about 350 KB per problem
 *   at n = 1024 and 40 steps);
 *   max_quad caps the per-problem quadrature M (0 = 65536; a problem whose
 *   rule asks for more reports CHEBDM_ERR_ARG in its status).  Allocates
 *   sum_p (k+m) ld_p^2 workspace elements (ld_p = round_up(n_p, 128)).
 * chebdm_batch_tune: the autotuner.  Times one product step for each
 *   candidate schedule on the plan's workspace (tile edge 64, 48 or 32 per
 *   size bucket n <= 256 / 512 / 768 / larger, a problem whose 48-tile grid
 *   would leave its workspace keeping 64; problems ordered by decreasing n or
 *   as given) and keeps the fastest.  Every candidate gives the same result
 *   bit for bit.  cache_path (nullable): a text file of
 *   "key value" lines; a matching key is applied without timing, a new result
 *   is appended.  report (nullable) receives a one-line summary.
 * chebdm_batch_mu_search: host arrays of count entries: dH[p], dD[p] (device
 *   float64 matrices, row-major), ldh[p], ldd[p], beta[p] > 0,
 *   0 < n_elec[p] < n[p]; outputs mu_out[p] and optional status_out[p]
 *   (chebdm_status of that problem), iters_out[p], trace_out[p] (tr D).
 *   Synchronises.  Returns the worst status (a negative one if any problem
 *   failed; the others are still valid).
 * chebdm_batch_info: k, m, products per problem, (problem, tile) items per
 *   product step, algorithmic flops of all products of one run.
 */
typedef struct chebdm_batch_ctx* chebdm_batch;

int chebdm_batch_create(chebdm_handle h, int32_t count, const int64_t* n, int32_t order,
                        const chebdm_opts* opts, int64_t max_quad, chebdm_batch* out);
int chebdm_batch_destroy(chebdm_batch b);
int chebdm_batch_tune(chebdm_batch b, const char* cache_path, char* report, int32_t report_len);
int chebdm_batch_mu_search(chebdm_batch b, const double* const* dH, const int64_t* ldh,
                           const double* beta, const double* n_elec, double* const* dD,
                           const int64_t* ldd, double* mu_out, int32_t* status_out,
                           int32_t* iters_out, double* trace_out);
int chebdm_batch_info(chebdm_batch b, int32_t* k, int32_t* m, int32_t* products_per_problem,
                      int64_t* tiles_per_step, double* flop_per_run);

/*
 * Moments-only runs: chebdm_batch_mu_search with dD == NULL (ldd ignored)
 * stops after the chemical-potential search (bounds, baby steps, ladder and
 * Gram moments, search); trace_out then receives the quadrature trace
 * t(mu~) at the returned mu.  It is captured as a graph of its own.
 *
 * chebdm_batch_set_search: how the per-problem search on the trace
 * function t(mu~) proceeds in later runs (the search itself is the
 * library's reading: the paper takes mu as an input; see chebdm_mu_search).
 *   mode 0  bisection on [-1, 1] (the default; what chebdm_mu_search does);
 *   mode 1  safeguarded Newton on [-1, 1] from mu~ = 0, with t' from the
 *           same quadrature (a step leaving the bracket is a bisection step);
 *   mode 2  learned start: the network (chebdm_mlp_*) with device weights dW
 *           (float32, chebdm_mlp_num_params() of them, read at every run,
 *           not copied; they must stay valid) maps the moments to a guess g;
 *           Newton steps run from g, each evaluated point becoming the low
 *           or the high end of the bracket, until both ends are evaluated
 *           points (then safeguarded Newton inside them) or the search
 *           converges.  A step with t' <= 0, outside [-1, 1] or further than
 *           delta from g, or no bracket after 8 evaluations, falls back to
 *           plain bisection between the ends found so far and whichever of
 *           -1, 1 is still unchecked (ERR_BRACKET if N_e is not inside).
 *           0 < delta <= 2.
 *   Every mode ends on |t - N_e| < tol, a bracket under 4 ulp or max_iter.
 *   Drops the captured graphs.  ERR_ARG on a bad mode, NULL dW or delta.
 * chebdm_batch_stats: after a run, per problem (each output nullable, host,
 *   count entries): evaluations of t (bracket checks included), whether the
 *   learned start converged or formed the bracket itself (0/1; 0 when it fell
 *   back), the scaled mu~ and beta' = beta a.
 * chebdm_batch_features: after a run, writes the network inputs of every
 *   problem to dfeat (device float32, count x 64 row-major): tau_1..tau_62
 *   divided by n, N_e / n, log(beta') / 4 (moments past the order are 0).
 */
int chebdm_batch_set_search(chebdm_batch b, int32_t mode, const float* dW, double delta);
int chebdm_batch_stats(chebdm_batch b, int32_t* evals, int32_t* learned, double* mu_s, double* beta_s);
int chebdm_batch_features(chebdm_batch b, float* dfeat);

/*
 * The learned chemical-potential network (not part of the paper: a start
 * guess for the library's chemical-potential search, which the paper does not
 * have: it takes mu as an input).  y = w3 . relu(W2 relu(W1 x + b1) + b2) + b3
 * with x in R^64, 256 units per hidden layer, float32.  Flat parameter
 * vector (device, float32): W1 (256 x 64 row-major), b1 (256), W2 (256 x 256),
 * b2 (256), w3 (256), b3 (1): chebdm_mlp_num_params() = 82689 floats.
 * All run on the handle's stream; the handle keeps a workspace of
 * 4 batch x 256 + 2 batch + 1 floats (grown on demand).
 *
 * chebdm_mlp_forward: dX (batch x 64), dY (batch).  Does not synchronise.
 * chebdm_mlp_backward: loss = mean_b (y_b - dT[b])^2 and its gradient with
 *   respect to every parameter into dGrad (same layout as dW, overwritten).
 *   loss_out (host, nullable): if given, the call synchronises and stores
 *   the loss.
 * chebdm_mlp_adam: one Adam update (Kingma and Ba) of dW with moment buffers
 *   dM, dV (zero before step 1), step >= 1, 0 <= beta1, beta2 < 1, lr > 0,
 *   eps >= 0.  Does not synchronise.
 */
int chebdm_mlp_num_params(void);
int chebdm_mlp_forward(chebdm_handle h, const float* dW, const float* dX, int32_t batch, float* dY);
int chebdm_mlp_backward(chebdm_handle h, const float* dW, const float* dX, const float* dT,
                        int32_t batch, float* dGrad, float* loss_out);
int chebdm_mlp_adam(chebdm_handle h, float* dW, const float* dGrad, float* dM, float* dV,
                    int32_t step, float lr, float beta1, float beta2, float eps);

/*
 * Launch timing.  While enabled, the library records a HIP event pair on its
 * stream around every launch of the matrix-product kernel (one pair per
 * grouped launch or batched product step), of the block-sum pass, of the
 * Gram contraction and of the chemical-potential search (DCT-III of the
 * moments and the search; in a batched run with the learned start, also the
 * feature and network passes); a batched run then executes eagerly on the
 * handle's stream instead of replaying its graph.
 * chebdm_profile_read synchronises the stream, sums the elapsed times since
 * the last read (or enable) and clears them.  Algorithmic work counted:
 *   gemm_flop   n^2 (n+1) per product (the n(n+1)/2 distinct outputs of a
 *               symmetric product, 2n flops each; padding and the discarded
 *               lower half of diagonal tiles are not counted);
 *   *_bytes     one read or write of each n x n matrix the pass streams
 *               (block sums: k-1 reads + m writes; Gram: nl + nt reads).
 * Not for use while the stream is being captured into a graph.
 */
typedef struct {
    int64_t gemm_launches;   /* launches of the product kernel                    */
    int64_t gemm_products;   /* products in them (a grouped launch holds several) */
    double gemm_ms;          /* summed launch durations                           */
    double gemm_flop;        /* algorithmic flops of those products               */
    int64_t combine_calls;
    double combine_ms, combine_bytes;
    int64_t gram_calls;
    double gram_ms, gram_bytes;
    int64_t search_calls;    /* DCT-III + mu search (+ network forward) passes   */
    double search_ms;
} chebdm_profile;

/* Turn launch timing on (enable != 0) or off; clears the counters. */
int chebdm_profile_enable(chebdm_handle h, int enable);

/* Synchronise, report the timings gathered since the last read, clear them. */
int chebdm_profile_read(chebdm_handle h, chebdm_profile* out);

#ifdef __cplusplus
}
#endif

#endif /* CHEBDM_H */
