// Host runtime behind the C ABI: argument checks, the baby/giant-step plan,
// the workspace, and the launch sequence of each entry point.
//
// Pipeline (Sec. II.B and III.B of the paper, readings noted in chebdm.h):
//   bounds -> T_1 = H~ -> [mu search: moments -> bisection] -> c_n -> block
//   coefficients -> baby steps (Algorithm 1 stages, one grouped launch per
//   stage) -> block sums R_l (one pass) -> m-1 giant steps -> D.
// Everything after the bounds runs on the device without host round trips;
// the host needs the bounds once, to size the quadrature from beta'.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "cheb_dev.h"
#include "ctx.h"
#include "internal.h"

using namespace chebdm;

namespace chebdm {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

// Opens a timed region on the handle's stream (no-op unless profiling is on).
int prof_begin(chebdm_handle h, int kind, int products, double flop, double bytes, size_t* idx) {
    *idx = (size_t)-1;
    if (!h->prof) return 0;
    if (h->ev_used == h->ev.size()) {
        chebdm_ctx::Ev e;
        HIP_TRY(hipEventCreate(&e.a));
        HIP_TRY(hipEventCreate(&e.b));
        h->ev.push_back(e);
    }
    chebdm_ctx::Ev& e = h->ev[h->ev_used];
    e.kind = kind;
    e.products = products;
    e.flop = flop;
    e.bytes = bytes;
    HIP_TRY(hipEventRecord(e.a, h->stream));
    *idx = h->ev_used++;
    return 0;
}

int prof_end(chebdm_handle h, size_t idx) {
    if (idx == (size_t)-1) return 0;
    HIP_TRY(hipEventRecord(h->ev[idx].b, h->stream));
    return 0;
}

// Algorithmic flops of one symmetric product: n(n+1)/2 distinct outputs, 2n flops each.
double sym_product_flop(int64_t n) { return (double)n * (double)n * (double)(n + 1); }

}  // namespace chebdm

namespace {



constexpr int64_t kMaxN = 65535;            // grid rows of the element-wise kernels
constexpr int64_t kSmallVec = 48 * 48 + 64; // c, block coefficients, tau
constexpr int64_t kPartialDoubles = 1024 * 48 * 48;  // Gram partials (>= Gershgorin partials)

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

struct Plan {
    int64_t n = 0, ld = 0;
    int order = 0, k = 1, m = 1, M = 0;
    int prec = CHEBDM_FP64, form = CHEBDM_GIANT_COMPOSITION, baby = CHEBDM_BABY_STAGES, ladder = CHEBDM_BABY_STAGES;
    int max_iter = 200;
    int search = CHEBDM_SEARCH_BISECTION;
    int damping = CHEBDM_DAMPING_NONE;
    int bounds = CHEBDM_BOUNDS_GERSHGORIN, lz_steps = 40;
    bool order_auto = true;   // baby-step and ladder orders are the library's choice
    int chains = 0;    // composition form: 0 library's choice, 1, 2 or 4 chains
    int split_h = 0;   // > 0: giant steps as two Clenshaw chains joined by T_h(T_k) (extra slot k + m)
    int split_q = 0;   // > 0: each half split again at q, joined by T_q(T_k) (extra slot k + m + 1)
    double lz_margin = 0.01;
    double tol = 1e-10;
    size_t elem = 8;
    int n_gemm = 0;
};

}  // namespace



namespace {

int set_device(chebdm_handle h) {
    HIP_TRY(hipSetDevice(h->device));
    return 0;
}

static_assert(sizeof(DevScalars) <= 64 * sizeof(double), "scalars must fit their 64-double slot");

size_t small_bytes_for(int64_t M) {
    const int64_t Mcap = M < 4096 ? 4096 : M;
    const int64_t doubles = 64 /*scalars*/ + 4 * kSmallVec + 48 * 48 + 64 + 3 * Mcap + kPartialDoubles;
    return (size_t)doubles * sizeof(double);
}

// Grows the small buffers.  The scalars carry over into a new allocation: the Gershgorin
// bounds written there by the bounds kernels are read back on the device by later kernels.
int ensure_small(chebdm_handle h, int64_t M) {
    if (h->small && M <= h->small_M) return 0;
    const int64_t Mcap = M < 4096 ? 4096 : M;
    const size_t bytes = small_bytes_for(M);
    void* fresh = nullptr;
    if (hipMalloc(&fresh, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(CHEBDM_ERR_OOM, "cannot allocate " + std::to_string(bytes) + " bytes of scalar workspace");
    }
    if (h->small) {
        HIP_TRY(hipMemcpyAsync(fresh, h->small, 64 * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        HIP_TRY(hipFree(h->small));
    }
    h->small = fresh;
    double* p = static_cast<double*>(h->small);
    h->scal = reinterpret_cast<DevScalars*>(p);
    p += 64;
    h->c = p; p += kSmallVec;
    h->coef = p; p += kSmallVec;
    h->tau = p; p += kSmallVec;
    h->trb = p; p += kSmallVec;
    h->gram = p; p += 48 * 48;
    h->trD = p; p += 64;
    h->ftab = p; p += Mcap;
    h->xtab = p; p += Mcap;
    h->w = p; p += Mcap;
    h->partial = p;
    h->small_bytes = bytes;
    h->small_M = Mcap;
    return 0;
}

int ensure_mats(chebdm_handle h, const Plan& pl, int64_t count) {
    const size_t bytes = (size_t)count * (size_t)pl.ld * (size_t)pl.ld * pl.elem;
    if (bytes > h->mats_bytes) {
        if (h->mats) {
            HIP_TRY(hipStreamSynchronize(h->stream));
            HIP_TRY(hipFree(h->mats));
            h->mats = nullptr;
            h->mats_bytes = 0;
        }
        if (hipMalloc(&h->mats, bytes) != hipSuccess) {
            h->mats = nullptr;
            (void)hipGetLastError();
            return fail(CHEBDM_ERR_OOM, "cannot allocate " + std::to_string(bytes) + " bytes of matrix workspace");
        }
        h->mats_bytes = bytes;
        h->lay_ld = -1;
    }
    // partial accumulators of K-sliced tail tiles of the products
    if (!h->gemm_scratch) {
        if (hipMalloc(&h->gemm_scratch, kGemmScratchBytes) != hipSuccess) {
            h->gemm_scratch = nullptr;
            (void)hipGetLastError();
            return fail(CHEBDM_ERR_OOM, "cannot allocate the product scratch");
        }
    }
    // The kernels rely on a zero padding outside each n x n block; a new
    // layout (n, leading dimension, element size or a larger count) is cleared once.
    if (h->lay_n != pl.n || h->lay_ld != pl.ld || h->lay_elem != pl.elem || h->lay_count < count) {
        HIP_TRY(hipMemsetAsync(h->mats, 0, bytes, h->stream));
        h->lay_n = pl.n;
        h->lay_ld = pl.ld;
        h->lay_elem = pl.elem;
        h->lay_count = count;
    }
    return 0;
}



// matrix slot s (0-based) of the workspace
void* slot(chebdm_handle h, const Plan& pl, int64_t s) {
    return static_cast<char*>(h->mats) + (size_t)s * (size_t)pl.ld * (size_t)pl.ld * pl.elem;
}

int read_scalars(chebdm_handle h) {
    HIP_TRY(hipMemcpyAsync(h->h_scal, h->scal, sizeof(DevScalars), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpyAsync(h->h_trD, h->trD, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return 0;
}

int quadrature_rule(int order, double beta_s) { return (int)quad_rule(order, beta_s); }

int check_opts(const chebdm_opts* o, Plan& pl) {
    chebdm_opts d;
    chebdm_default_opts(&d);
    if (!o) o = &d;
    if (o->prec < CHEBDM_FP64 || o->prec > CHEBDM_BF16X6) return fail(CHEBDM_ERR_ARG, "unknown precision");
    if (o->giant_form < CHEBDM_GIANT_COMPOSITION || o->giant_form > CHEBDM_GIANT_FOUR_CHAINS)
        return fail(CHEBDM_ERR_ARG, "unknown giant-step form");
    if (o->giant_form == CHEBDM_GIANT_POWER && o->prec != CHEBDM_FP64)
        return fail(CHEBDM_ERR_UNSUPPORTED,
                    "the power form is float64 only: its coefficients grow like 2^m |c|");
    if (o->k_override < 0 || o->n_quad < 0 || o->max_iter < 0 || !(o->tol >= 0.0))
        return fail(CHEBDM_ERR_ARG, "negative option");
    if (o->baby_steps < CHEBDM_BABY_AUTO || o->baby_steps > CHEBDM_BABY_ODD_CHAINS)
        return fail(CHEBDM_ERR_ARG, "unknown baby-step schedule");
    if (o->search != CHEBDM_SEARCH_BISECTION && o->search != CHEBDM_SEARCH_NEWTON)
        return fail(CHEBDM_ERR_ARG, "unknown mu search");
    pl.search = o->search;
    if (o->damping != CHEBDM_DAMPING_NONE && o->damping != CHEBDM_DAMPING_JACKSON)
        return fail(CHEBDM_ERR_ARG, "unknown damping");
    pl.damping = o->damping;
    if (o->bounds != CHEBDM_BOUNDS_GERSHGORIN && o->bounds != CHEBDM_BOUNDS_LANCZOS)
        return fail(CHEBDM_ERR_ARG, "unknown bounds method");
    if (o->lanczos_steps < 0 || o->lanczos_steps > kMaxLanczosSteps)
        return fail(CHEBDM_ERR_ARG, "lanczos_steps must be in [0, 128]");
    if (!(o->bounds_margin >= 0.0) || !std::isfinite(o->bounds_margin))
        return fail(CHEBDM_ERR_ARG, "bounds_margin must be finite and >= 0");
    pl.bounds = o->bounds;
    pl.lz_steps = o->lanczos_steps ? o->lanczos_steps : 40;
    pl.lz_margin = o->bounds_margin > 0.0 ? o->bounds_margin : 0.01;
    // Float32 baby steps go in odd chains: the stages lose to the sequential order on loose
    // bounds (float32 CPU model, N = 1000, Gershgorin: 1.5e-4 against 2.4e-7), where T_1 and
    // every odd T_s are small; chains of step 3, 5 or 7 match the sequential order there and
    // every order agrees on tight bounds.  The split-bf16 products stay sequential (their
    // chains double the error, and they sit closer to their tolerance).
    pl.order_auto = o->baby_steps == CHEBDM_BABY_AUTO;
    pl.baby = o->baby_steps != CHEBDM_BABY_AUTO
                  ? o->baby_steps
                  : (o->prec == CHEBDM_FP64 ? CHEBDM_BABY_STAGES
                                            : (o->prec == CHEBDM_FP32 ? CHEBDM_BABY_ODD_CHAINS : CHEBDM_BABY_SEQUENTIAL));
    // The ladder T_{lk} = T_l(T_k) multiplies O(1)-norm matrices in either order, and with
    // float32 products the stages cost it no accuracy (moments at N = 1000 within a factor of 2
    // of the sequential order's; the baby steps' sequential order keeps its edge only because it
    // multiplies by T_1, whose norm is far below 1 on loose bounds).  The split-bf16 products
    // lose about an order of magnitude in the moments when staged, so they keep the sequential
    // ladder.
    pl.ladder = o->baby_steps != CHEBDM_BABY_AUTO
                    ? o->baby_steps
                    : (o->prec == CHEBDM_FP64 || o->prec == CHEBDM_FP32 ? CHEBDM_BABY_STAGES
                                                                         : CHEBDM_BABY_SEQUENTIAL);
    pl.prec = o->prec;
    pl.form = o->giant_form == CHEBDM_GIANT_POWER ? CHEBDM_GIANT_POWER : CHEBDM_GIANT_COMPOSITION;
    pl.chains = o->giant_form == CHEBDM_GIANT_ONE_CHAIN    ? 1
                : o->giant_form == CHEBDM_GIANT_TWO_CHAINS ? 2
                : o->giant_form == CHEBDM_GIANT_FOUR_CHAINS ? 4
                                                            : 0;
    pl.elem = o->prec == CHEBDM_FP64 ? 8 : 4;
    pl.max_iter = o->max_iter ? o->max_iter : 200;
    pl.tol = o->tol > 0.0 ? o->tol : 1e-10;
    pl.M = o->n_quad;
    pl.k = o->k_override;
    return 0;
}

int plan_split(Plan& pl) {
    const int64_t ncoef = (int64_t)pl.order + 1;
    int64_t k = pl.k;
    if (k <= 0) {
        k = (int64_t)std::sqrt((double)ncoef);
        while (k * k < ncoef) ++k;
        while (k > 1 && (k - 1) * (k - 1) >= ncoef) --k;
    }
    const int64_t m = (ncoef + k - 1) / k;
    if (k > kMaxBlocks || m > kMaxBlocks)
        return fail(CHEBDM_ERR_ARG, "order " + std::to_string(pl.order) + " with k=" + std::to_string(k) +
                                        " needs more than 48 baby steps or blocks");
    pl.k = (int)k;
    pl.m = (int)m;
    // Float32 past k = 24 (orders from 576 on): sequential baby steps and ladder.  The odd
    // chains multiply by T_s with s up to 7, whose rounding compounds over the 45 steps of
    // k = 46: N = 5000, order 2048, beta' ~ 1e4, max|D - D_oracle| 3.5e-5 with the odd chains and
    // the staged ladder against 7.6e-6 sequentially.  There every product fills the chip on its
    // own, so the sequential order costs little.
    if (pl.order_auto && pl.prec == CHEBDM_FP32 && pl.k > 24) {
        pl.baby = CHEBDM_BABY_SEQUENTIAL;
        pl.ladder = CHEBDM_BABY_SEQUENTIAL;
    }
    return 0;
}

int validate_matrix(const void* dH, int64_t n, int64_t ldh) {
    if (!dH) return fail(CHEBDM_ERR_ARG, "H is NULL");
    if (n < 1 || n > kMaxN) return fail(CHEBDM_ERR_ARG, "n must be in [1, 65535]");
    if (ldh < n) return fail(CHEBDM_ERR_ARG, "leading dimension smaller than n");
    return 0;
}

int lanczos_on_device(chebdm_handle h, const double* dH, int64_t n, int64_t ldh, int steps, double margin,
                      uint64_t seed);

// Bounds: the caller's, or computed here (one read-back): Gershgorin's, then with
// CHEBDM_BOUNDS_LANCZOS the Lanczos bounds inside them.
int resolve_bounds(chebdm_handle h, const double* dH, int64_t n, int64_t ldh, double& emin, double& emax,
                   const Plan* pl = nullptr) {
    if (std::isnan(emin) || std::isnan(emax)) {
        CHECK(ensure_small(h, 0));
        HIP_TRY(launch_gershgorin(dH, n, ldh, h->partial, kPartialDoubles, h->scal, h->stream));
        if (pl && pl->bounds == CHEBDM_BOUNDS_LANCZOS)
            CHECK(lanczos_on_device(h, dH, n, ldh, pl->lz_steps, pl->lz_margin, 0));
        CHECK(read_scalars(h));
        if (h->h_scal->nonfinite) return fail(CHEBDM_ERR_NONFINITE, "H holds NaN or Inf");
        emin = h->h_scal->emin;
        emax = h->h_scal->emax;
    }
    if (!std::isfinite(emin) || !std::isfinite(emax) || emax < emin)
        return fail(CHEBDM_ERR_ARG, "bounds must be finite with emin <= emax");
    return 0;
}

// Library's choice between one and two giant-step chains: two wherever they can be used.
// Measured (mu search + D, order 512, DM/s one -> two chains): N = 1000 float64 407 -> 414,
// float32 420 -> 436, split-bf16 356 -> 386; N = 2000 float64 82.6 -> 82.8, float32 107.8 ->
// 111.2, split-bf16 164 -> 179; N = 4000 float64 13.70 -> 13.70, float32 27.12 -> 27.04,
// split-bf16 48.5 -> 49.6.
bool two_chains_pay(const Plan& pl) { return pl.n > 0; }

int plan_quadrature(Plan& pl, double beta, double emin, double emax) {
    const double beta_s = beta * 0.5 * (emax - emin);
    if (pl.M <= 0) pl.M = quadrature_rule(pl.order, beta_s);
    if (pl.M <= 0) return fail(CHEBDM_ERR_ARG, "beta' too large for the quadrature rule");
    if (pl.M < pl.order + 1) return fail(CHEBDM_ERR_ARG, "n_quad must be at least order + 1");
    if (pl.M > (1 << 26)) return fail(CHEBDM_ERR_ARG, "n_quad above 2^26");
    return 0;
}

// Split point of the two-chain giant steps, or 0 for one chain.  Two chains need T_h(T_k), which
// only the mu search's moment ladder provides, and m >= 4; the library's choice takes them
// where one product per launch leaves the chip underfilled.
int two_chain_split(const Plan& pl, bool ladder_and_density) {
    if (pl.form != CHEBDM_GIANT_COMPOSITION || !ladder_and_density || pl.m < 4 || pl.chains == 1) return 0;
    if (pl.chains == 0 && !two_chains_pay(pl)) return 0;
    return (pl.m + 1) / 2;
}

// Library's choice between two and four chains where both are possible: four while one product
// holds less than a full round of 64-tiles (1024: 256 CUs at one wavefront per SIMD), where two
// products per launch still leave the chip part idle.  Measured (mu search + D, order 512, DM/s
// two -> four chains): N = 1000 float64 412 -> 432, float32 515 -> 543, split-bf16 387 -> 423;
// N = 2000 float64 87.3 -> 89.4, float32 140.7 -> 146.4, split-bf16 179.8 -> 189.5; N = 4000
// (2016 tiles per product) within noise: 13.75 -> 13.71, 27.05 -> 27.07, 52.6 -> 52.4.
bool four_chains_pay(const Plan& pl) {
    const int64_t t = round_up(pl.n, 128) / 64;
    return t * (t + 1) / 2 < 1024;
}

// Second split point of the four-chain giant steps, or 0: both halves of the two chains (blocks
// 0..h-1 and h..m-1, the second no longer than the first) split at q = ceil(h/2).  Needs m >= 8
// (q >= 2; the last chain may be a single block) and T_q(T_k) from the ladder.
int four_chain_split(const Plan& pl, int split_h) {
    if (split_h == 0 || pl.m < 8 || pl.chains == 1 || pl.chains == 2) return 0;
    if (pl.chains == 0 && !four_chains_pay(pl)) return 0;
    return (split_h + 1) / 2;
}

// Slots the giant-step chains keep beyond the k + m of the plan: T_h(T_k), and T_q(T_k).
int extra_chain_slots(const Plan& pl) { return (pl.split_h > 0 ? 1 : 0) + (pl.split_q > 0 ? 1 : 0); }

// ---------------------------------------------------------------- GEMM helper

struct Chain {
    chebdm_handle h;
    const Plan& pl;
    int* n_gemm;
    GemmBatch<double> b64;
    GemmBatch<float> b32;

    Chain(chebdm_handle hh, const Plan& p, int* ng) : h(hh), pl(p), n_gemm(ng) {
        b64.count = 0;
        b32.count = 0;
    }
    // Out = alpha A B + beta C + gamma E + delta I
    void add(const void* A, const void* B, const void* C, double beta, const void* E, double gamma,
             double alpha, double delta, void* Out, int64_t ld_out, int out_f64) {
        if (pl.elem == 8) {
            GemmDesc<double>& d = b64.d[b64.count++];
            d = GemmDesc<double>{(const double*)A, (const double*)B, (const double*)C, (const double*)E, Out,
                                 ld_out, alpha, beta, gamma, delta, out_f64, 0};
        } else {
            GemmDesc<float>& d = b32.d[b32.count++];
            d = GemmDesc<float>{(const float*)A, (const float*)B, (const float*)C, (const float*)E, Out,
                                ld_out, alpha, beta, gamma, delta, out_f64, 0};
        }
        ++*n_gemm;
    }
    int flush() {
        const int cnt = pl.elem == 8 ? b64.count : b32.count;
        if (cnt == 0) return 0;
        size_t ev;
        CHECK(prof_begin(h, PROF_GEMM, cnt, cnt * sym_product_flop(pl.n), 0.0, &ev));
        hipError_t e = hipSuccess;
        if (pl.elem == 8) e = launch_gemm_f64(b64, pl.n, pl.ld, h->stream, h->gemm_scratch,
                                              h->gemm_scratch ? kGemmScratchBytes : 0);
        else e = launch_gemm_f32(b32, pl.n, pl.ld,
                                 pl.prec == CHEBDM_BF16X6 ? 2 : (pl.prec == CHEBDM_BF16X3 ? 1 : 0), h->stream,
                                 h->gemm_scratch, h->gemm_scratch ? kGemmScratchBytes : 0);
        b64.count = 0;
        b32.count = 0;
        HIP_TRY(e);
        CHECK(prof_end(h, ev));
        return 0;
    }
};

// T_i for i >= 1 lives in slot i-1.
void* tslot(chebdm_handle h, const Plan& pl, int i) { return slot(h, pl, i - 1); }
// R_l lives in slot k + l.
void* rslot(chebdm_handle h, const Plan& pl, int l) { return slot(h, pl, pl.k + l); }

// Step s of the odd-chain schedule for P_2..P_K: the odd s >= 3 with the fewest launches when
// P_2..P_s take s - 1 one-product launches, plus ceil((K - s) / s) rounds of s; ties go to the
// smaller s.  Returns 0 (plain sequential order) when K is too small for a chain round.
int odd_chain_step(int K) {
    int best = 0, best_launches = K - 1;
    for (int s = 3; s < K; s += 2) {
        const int launches = (s - 1) + (K - s + s - 1) / s;
        if (launches < best_launches) {
            best = s;
            best_launches = launches;
        }
    }
    return best;
}

// Baby steps T_2..T_k in the stages of Algorithm 1: stage 1 makes T_2; stage
// s >= 2 makes T_{2^{s-2}+i} and T_{2^{s-1}+i} from already known T's.  The
// products of one stage are independent and go out as one grouped launch.
// ---------------------------------------------------------------- graph replay

// Everything a captured device sequence depends on: if two calls agree on all of it, every
// kernel argument of their sequences agrees, and the first call's graph can be replayed.
struct ReplayKey {
    int32_t kind, order, k, m, prec, form, baby, ladder, search, max_iter, bounds_on_device, damping, split_h, split_q;
    int64_t n, ld, ldh, ldd, M;
    const void *dH, *dD, *mats, *small;
    double tol, beta, x, emin, emax;   // x: n_elec (mu search) or mu (density)
};

std::vector<char> replay_key(int kind, const Plan& pl, chebdm_handle h, const double* dH, int64_t ldh,
                             const double* dD, int64_t ldd, double beta, double x, bool bounds_on_device,
                             double emin, double emax) {
    ReplayKey k;
    std::memset(&k, 0, sizeof(k));   // padding too: keys are compared byte by byte
    k.kind = kind;
    k.order = pl.order;
    k.k = pl.k;
    k.m = pl.m;
    k.prec = pl.prec;
    k.form = pl.form;
    k.split_h = pl.split_h;
    k.split_q = pl.split_q;
    k.baby = pl.baby;
    k.ladder = pl.ladder;
    k.search = pl.search;
    k.max_iter = pl.max_iter;
    k.damping = pl.damping;
    k.bounds_on_device = bounds_on_device ? 1 : 0;
    k.n = pl.n;
    k.ld = pl.ld;
    k.ldh = ldh;
    k.ldd = ldd;
    k.M = pl.M;
    k.dH = dH;
    k.dD = dD;
    k.mats = h->mats;
    k.small = h->small;
    k.tol = pl.tol;
    k.beta = beta;
    k.x = x;
    if (!bounds_on_device) {
        k.emin = emin;
        k.emax = emax;
    }
    std::vector<char> v(sizeof(k));
    std::memcpy(v.data(), &k, sizeof(k));
    return v;
}

void drop_replay(chebdm_ctx::Replay& r) {
    if (r.exec) (void)hipGraphExecDestroy(r.exec);
    if (r.graph) (void)hipGraphDestroy(r.graph);
    r.exec = nullptr;
    r.graph = nullptr;
    r.key.clear();
}

// Runs body() - launches only, all on h->stream - either eagerly (launch timing on) or as a
// graph: captured on the handle's own stream on first use, replayed on h->stream while the
// key matches.  The replay is ordered after everything already queued on h->stream.
// *products: the body's product count (kept with the graph for replays).
template <class Body>
int run_replayed(chebdm_handle h, int slot, const std::vector<char>& key, int* products, Body body) {
    if (h->prof) return body();
    chebdm_ctx::Replay& r = h->replay[slot];
    if (!r.exec || r.key != key) {
        drop_replay(r);
        if (!h->cap) HIP_TRY(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
        hipStream_t user = h->stream;
        h->stream = h->cap;
        const int rc = body();
        h->stream = user;
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(h->cap, &g);
        if (rc < 0) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        HIP_TRY(ec);
        r.graph = g;
        const hipError_t ei = hipGraphInstantiate(&r.exec, g, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            drop_replay(r);
            HIP_TRY(ei);
        }
        r.key = key;
        r.products = *products;
    }
    *products = r.products;
    HIP_TRY(hipGraphLaunch(r.exec, h->stream));
    return 0;
}

// ---------------------------------------------------------------- Lanczos bounds

struct LanczosKey {
    const void *dH, *lz, *small;
    int64_t n, ldh;
    int32_t steps, pad;
    double margin;
    uint64_t seed;
};

int ensure_lanczos(chebdm_handle h, int64_t n, int steps) {
    const int64_t need = lanczos_work_doubles(n, steps);
    if (need <= h->lz_doubles) return 0;
    drop_replay(h->replay[3]);
    if (h->lz) HIP_TRY(hipFree(h->lz));
    h->lz = nullptr;
    h->lz_doubles = 0;
    if (hipMalloc(&h->lz, sizeof(double) * (size_t)need) != hipSuccess) {
        h->lz = nullptr;
        (void)hipGetLastError();
        return fail(CHEBDM_ERR_OOM, "cannot allocate the Lanczos workspace");
    }
    h->lz_doubles = need;
    return 0;
}

// Lanczos bounds into h->scal (which holds the Gershgorin bounds); the launch sequence is
// captured once per argument set and replayed.
int lanczos_on_device(chebdm_handle h, const double* dH, int64_t n, int64_t ldh, int steps, double margin,
                      uint64_t seed) {
    const int k = (int)std::min<int64_t>(steps, n);
    CHECK(ensure_lanczos(h, n, k));
    LanczosKey lk;
    std::memset(&lk, 0, sizeof(lk));
    lk.dH = dH;
    lk.lz = h->lz;
    lk.small = h->small;
    lk.n = n;
    lk.ldh = ldh;
    lk.steps = k;
    lk.margin = margin;
    lk.seed = seed;
    std::vector<char> key(sizeof(lk));
    std::memcpy(key.data(), &lk, sizeof(lk));
    int unused = 0;
    return run_replayed(h, 3, key, &unused, [&]() -> int {
        HIP_TRY(launch_lanczos(dH, n, ldh, k, margin, seed, h->lz, h->scal, h->stream));
        return 0;
    });
}

// P_2(Y) .. P_K(Y) from P_1 = Y and P_0 = I for the Chebyshev polynomials P_i = T_i of a
// symmetric Y, where slot(i) holds P_i (i >= 1).  Sequential: P_{i+1} = 2 Y P_i - P_{i-1}.
// Stages (Algorithm 1, Sec. III.B): stage s forms P_{v+1..2v} (v = 2^{s-1}) from P_1..P_v by
// P_{i+u} = 2 P_i P_u - P_{i-u} and P_{i+v} = 2 P_v P_i - P_{v-i} (u = v/2, u < i <= v); the
// products of a stage are independent and go out as one grouped launch.
// Odd chains: P_2..P_s (by the same rule with a smaller step, or sequentially), then
// P_{i+s} = 2 P_s P_i - P_{|i-s|} for the s products of each round (their operands come from
// earlier rounds).
template <class Slot>
int chebyshev_powers(Chain& ch, const Plan& pl, Slot slot, int K, int sched) {
    if (K < 2) return 0;
    const int cs = sched == CHEBDM_BABY_ODD_CHAINS ? odd_chain_step(K) : 0;
    if (sched == CHEBDM_BABY_SEQUENTIAL || sched == CHEBDM_BABY_ODD_CHAINS) {
        if (cs > 0) {
            CHECK(chebyshev_powers(ch, pl, slot, cs, CHEBDM_BABY_ODD_CHAINS));   // P_2..P_s
        } else {
            for (int i = 1; i < K; ++i) {
                ch.add(slot(1), slot(i), i == 1 ? nullptr : slot(i - 1), -1.0, nullptr, 0.0, 2.0,
                       i == 1 ? -1.0 : 0.0, slot(i + 1), pl.ld, 0);
                CHECK(ch.flush());
            }
        }
        for (int g0 = cs + 1; cs > 0 && g0 <= K; g0 += cs) {
            for (int i = g0; i < g0 + cs && i <= K; ++i) {
                const int j = i - cs, r = j > cs ? j - cs : cs - j;
                ch.add(slot(cs), slot(j), r == 0 ? nullptr : slot(r), -1.0, nullptr, 0.0, 2.0, r == 0 ? -1.0 : 0.0,
                       slot(i), pl.ld, 0);
            }
            CHECK(ch.flush());
        }
        return 0;
    }
    // stage 1: P_2 = 2 P_1 P_1 - P_0
    ch.add(slot(1), slot(1), nullptr, 0.0, nullptr, 0.0, 2.0, -1.0, slot(2), pl.ld, 0);
    CHECK(ch.flush());
    for (int s = 2;; ++s) {
        const int u = 1 << (s - 2), v = 1 << (s - 1);
        if (u + 1 + u > K && v + u + 1 > K) break;
        for (int i = u + 1; i <= v; ++i)
            if (i + u <= K) {
                const int r = i - u;
                ch.add(slot(i), slot(u), r == 0 ? nullptr : slot(r), -1.0, nullptr, 0.0, 2.0, r == 0 ? -1.0 : 0.0,
                       slot(i + u), pl.ld, 0);
            }
        for (int i = u + 1; i <= v; ++i)
            if (i + v <= K) {
                const int r = v - i;
                ch.add(slot(v), slot(i), r == 0 ? nullptr : slot(r), -1.0, nullptr, 0.0, 2.0, r == 0 ? -1.0 : 0.0,
                       slot(i + v), pl.ld, 0);
            }
        CHECK(ch.flush());
        if (v >= K) break;
    }
    return 0;
}

int baby_steps(chebdm_handle h, const Plan& pl, int* n_gemm) {
    Chain ch(h, pl, n_gemm);
    return chebyshev_powers(ch, pl, [&](int i) -> void* { return tslot(h, pl, i); }, pl.k, pl.baby);
}

// Ladder T_{2k}, ..., T_{lmax k} (T_{lk} in R slot l-2) and the moments tau_0..tau_L.
int moments_on_device(chebdm_handle h, const Plan& pl, int* n_gemm) {
    const int k = pl.k, L = pl.order;
    int lmax = (L >= 1) ? (L - 1) / k : 0;
    if (lmax > pl.m - 1) lmax = pl.m - 1;
    // T_{lk} lives in R slot l - 2 (overwritten later by the block sums), except T_{hk} of a
    // split giant-step chain, which is kept in slot k + m
    auto lptr = [&](int l) -> void* {
        if (l == 1) return tslot(h, pl, k);
        if (pl.split_h > 0 && l == pl.split_h) return slot(h, pl, (int64_t)k + pl.m);
        if (pl.split_q > 0 && l == pl.split_q) return slot(h, pl, (int64_t)k + pl.m + 1);
        return rslot(h, pl, l - 2);
    };
    // the ladder T_{lk} = T_l(T_k) is the same Chebyshev recurrence in Y = T_k, with a schedule
    // of its own (stage-parallel unless the caller asks for the sequential order)
    Chain ch(h, pl, n_gemm);
    CHECK(chebyshev_powers(ch, pl, lptr, lmax, pl.ladder));
    const int64_t stride = pl.ld * pl.ld;
    HIP_TRY(launch_traces(tslot(h, pl, 1), stride, k, pl.n, pl.ld, pl.elem == 8, h->trb, h->stream));
    if (lmax >= 1) {
        std::vector<const void*> lm(lmax), tm(k);
        for (int l = 1; l <= lmax; ++l) lm[l - 1] = lptr(l);
        for (int i = 1; i <= k; ++i) tm[i - 1] = tslot(h, pl, i);
        const int64_t nelem = pl.n * pl.ld;
        size_t ev;
        CHECK(prof_begin(h, PROF_GRAM, 0, 0.0, (double)(lmax + k) * pl.n * pl.n * pl.elem, &ev));
        if (pl.elem == 8)
            HIP_TRY(launch_gram<double>((const double* const*)lm.data(), lmax, (const double* const*)tm.data(), k,
                                        nelem, h->partial, kPartialDoubles, h->gram, h->stream));
        else
            HIP_TRY(launch_gram<float>((const float* const*)lm.data(), lmax, (const float* const*)tm.data(), k,
                                       nelem, h->partial, kPartialDoubles, h->gram, h->stream));
        CHECK(prof_end(h, ev));
    }
    HIP_TRY(launch_assemble_moments(h->trb, h->gram, k, pl.m, L, pl.n, h->tau, h->stream));
    return 0;
}

// Block sums R_l (or S_j) and the giant steps; writes D (ldd) and its trace.
int giant_steps(chebdm_handle h, const Plan& pl, double* dD, int64_t ldd, int* n_gemm) {
    const int k = pl.k, m = pl.m;
    const int64_t stride = pl.ld * pl.ld;
    size_t ev;
    CHECK(prof_begin(h, PROF_COMBINE, 0, 0.0, (double)(k - 1 + m) * pl.n * pl.n * pl.elem, &ev));
    if (pl.elem == 8)
        HIP_TRY(launch_combine<double>((const double*)tslot(h, pl, 1), stride, k, m, h->coef,
                                       (double*)rslot(h, pl, 0), pl.n, pl.ld, h->stream));
    else
        HIP_TRY(launch_combine<float>((const float*)tslot(h, pl, 1), stride, k, m, h->coef,
                                      (float*)rslot(h, pl, 0), pl.n, pl.ld, h->stream));
    CHECK(prof_end(h, ev));
    if (m == 1) {
        HIP_TRY(launch_copy_out(rslot(h, pl, 0), pl.elem == 8, pl.ld, pl.n, dD, ldd, h->stream));
    } else {
        void* Y = k >= 1 ? tslot(h, pl, k) : nullptr;
        Chain ch(h, pl, n_gemm);
        if (pl.form == CHEBDM_GIANT_COMPOSITION && pl.split_q > 0) {
            // four Clenshaw chains in Y = T_k, advanced together (up to four products per launch):
            // blocks [0, q), [q, h), [h, h+q), [h+q, m) after both splits; then
            // U_A = S_0 + T_q(Y) S_q and U_B = S_h + T_q(Y) S_{h+q} in one launch (in place in
            // R slots 0 and h), then D = U_A + T_h(Y) U_B.
            const int hs = pl.split_h, qs = pl.split_q;
            const int base[4] = {0, qs, hs, hs + qs};
            const int len[4] = {qs, hs - qs, qs, m - hs - qs};
            auto step = [&](int b, int n_l, int l) {
                const void* b2 = (l + 2 <= n_l - 1) ? rslot(h, pl, b + l + 2) : nullptr;
                const double a = l >= 1 ? 2.0 : 1.0;
                ch.add(Y, rslot(h, pl, b + l + 1), b2, -1.0, rslot(h, pl, b + l), 1.0, a, 0.0, rslot(h, pl, b + l),
                       pl.ld, 0);
            };
            for (int t = 0; t < qs - 1; ++t) {
                for (int c = 0; c < 4; ++c)
                    if (t < len[c] - 1) step(base[c], len[c], len[c] - 2 - t);
                CHECK(ch.flush());
            }
            const void* Tq = slot(h, pl, (int64_t)k + m + 1);
            ch.add(Tq, rslot(h, pl, qs), nullptr, 0.0, rslot(h, pl, 0), 1.0, 1.0, 0.0, rslot(h, pl, 0), pl.ld, 0);
            ch.add(Tq, rslot(h, pl, hs + qs), nullptr, 0.0, rslot(h, pl, hs), 1.0, 1.0, 0.0, rslot(h, pl, hs), pl.ld,
                   0);
            CHECK(ch.flush());
            ch.add(slot(h, pl, (int64_t)k + m), rslot(h, pl, hs), nullptr, 0.0, rslot(h, pl, 0), 1.0, 1.0, 0.0, dD,
                   ldd, 1);
            CHECK(ch.flush());
        } else if (pl.form == CHEBDM_GIANT_COMPOSITION && pl.split_h > 0) {
            // two Clenshaw chains in Y = T_k, advanced together (two products per launch):
            // S_A = sum_{l<h} T_l(Y) R''_l over R slots 0..h-1 and S_B = sum_{j<m-h} T_j(Y) R'_j
            // over R slots h..m-1 (blocks rearranged by launch_split_blocks), then
            // D = S_A + T_h(Y) S_B with T_h(Y) = T_{hk} kept from the ladder.
            const int hs = pl.split_h;
            const int la = hs, lb = m - hs;   // chain lengths (terms)
            auto step = [&](int base, int len, int l) {   // Clenshaw step l of the chain at R slot base
                const void* b2 = (l + 2 <= len - 1) ? rslot(h, pl, base + l + 2) : nullptr;
                const double a = l >= 1 ? 2.0 : 1.0;
                ch.add(Y, rslot(h, pl, base + l + 1), b2, -1.0, rslot(h, pl, base + l), 1.0, a, 0.0,
                       rslot(h, pl, base + l), pl.ld, 0);
            };
            for (int t = 0; t < la - 1; ++t) {
                step(0, la, la - 2 - t);
                if (t < lb - 1) step(hs, lb, lb - 2 - t);
                CHECK(ch.flush());
            }
            ch.add(slot(h, pl, (int64_t)k + m), rslot(h, pl, hs), nullptr, 0.0, rslot(h, pl, 0), 1.0, 1.0, 0.0, dD,
                   ldd, 1);
            CHECK(ch.flush());
        } else if (pl.form == CHEBDM_GIANT_COMPOSITION) {
            // Clenshaw over l with Y = T_k: B_{m-1} = R_{m-1};
            // B_l = R_l + 2 Y B_{l+1} - B_{l+2} (in place in R_l); D = R_0 + Y B_1 - B_2.
            for (int l = m - 2; l >= 1; --l) {
                const void* b2 = (l + 2 <= m - 1) ? rslot(h, pl, l + 2) : nullptr;
                ch.add(Y, rslot(h, pl, l + 1), b2, -1.0, rslot(h, pl, l), 1.0, 2.0, 0.0, rslot(h, pl, l), pl.ld, 0);
                CHECK(ch.flush());
            }
            const void* b2 = (m >= 3) ? rslot(h, pl, 2) : nullptr;
            ch.add(Y, rslot(h, pl, 1), b2, -1.0, rslot(h, pl, 0), 1.0, 1.0, 0.0, dD, ldd, 1);
            CHECK(ch.flush());
        } else {
            // Horner with T_k (eq. "ansatz"): R = S_{m-1}; R <- S_j + T_k R, j = m-2..0.
            for (int j = m - 2; j >= 1; --j) {
                ch.add(Y, rslot(h, pl, j + 1), nullptr, 0.0, rslot(h, pl, j), 1.0, 1.0, 0.0, rslot(h, pl, j), pl.ld, 0);
                CHECK(ch.flush());
            }
            ch.add(Y, rslot(h, pl, 1), nullptr, 0.0, rslot(h, pl, 0), 1.0, 1.0, 0.0, dD, ldd, 1);
            CHECK(ch.flush());
        }
    }
    HIP_TRY(launch_trace_f64(dD, pl.n, ldd, h->trD, h->stream));
    return 0;
}

void fill_info(chebdm_info* info, const Plan& pl, double emin, double emax, double mu, double trace,
               double trace_err, int iters, int status) {
    if (!info) return;
    info->k = pl.k;
    info->m = pl.m;
    info->n_gemm = pl.n_gemm;
    info->n_quad = pl.M;
    info->iters = iters;
    info->status = status;
    info->emin = emin;
    info->emax = emax;
    info->mu = mu;
    info->trace = trace;
    info->trace_err = trace_err;
}

double fermi_energy(double e, double beta, double mu) { return 1.0 / (1.0 + std::exp(beta * (e - mu))); }

}  // namespace

// =================================================================== C ABI

extern "C" {

void chebdm_default_opts(chebdm_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->prec = CHEBDM_FP64;
    o->giant_form = CHEBDM_GIANT_COMPOSITION;
    o->baby_steps = CHEBDM_BABY_AUTO;
    o->max_iter = 200;
    o->tol = 1e-10;
}

int chebdm_abi_version(void) { return CHEBDM_ABI_VERSION; }

const char* chebdm_last_error(void) { return g_last_error.c_str(); }

int chebdm_create(chebdm_handle* out, int device, void* stream) {
    if (!out) return fail(CHEBDM_ERR_ARG, "out is NULL");
    *out = nullptr;
    int count = 0;
    HIP_TRY(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(CHEBDM_ERR_ARG, "no such HIP device");
    HIP_TRY(hipSetDevice(device));
    CHECK(noalloc_setup(device));
    chebdm_ctx* h = new (std::nothrow) chebdm_ctx();
    if (!h) return fail(CHEBDM_ERR_OOM, "cannot allocate handle");
    h->device = device;
    h->stream = static_cast<hipStream_t>(stream);
    if (hipHostMalloc((void**)&h->h_scal, sizeof(DevScalars) + 64, hipHostMallocDefault) != hipSuccess) {
        delete h;
        return fail(CHEBDM_ERR_OOM, "cannot allocate pinned host memory");
    }
    h->h_trD = reinterpret_cast<double*>(reinterpret_cast<char*>(h->h_scal) + sizeof(DevScalars) + 8);
    g_last_error.clear();
    *out = h;
    return CHEBDM_OK;
}

int chebdm_destroy(chebdm_handle h) {
    if (!h) return CHEBDM_OK;
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);
    for (auto& e : h->ev) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    for (auto& r : h->replay) drop_replay(r);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    if (h->mats) (void)hipFree(h->mats);
    if (h->small) (void)hipFree(h->small);
    if (h->lz) (void)hipFree(h->lz);
    if (h->gemm_scratch) (void)hipFree(h->gemm_scratch);
    if (h->mlp_work) (void)hipFree(h->mlp_work);
    if (h->h_scal) (void)hipHostFree(h->h_scal);
    delete h;
    return CHEBDM_OK;
}

int chebdm_set_stream(chebdm_handle h, void* stream) {
    if (!h) return fail(CHEBDM_ERR_ARG, "handle is NULL");
    h->stream = static_cast<hipStream_t>(stream);
    return CHEBDM_OK;
}

int chebdm_bounds(chebdm_handle h, const double* dH, int64_t n, int64_t ldh, double* emin, double* emax) {
    if (!h || !emin || !emax) return fail(CHEBDM_ERR_ARG, "NULL argument");
    CHECK(validate_matrix(dH, n, ldh));
    CHECK(set_device(h));
    double lo = NAN, hi = NAN;
    CHECK(resolve_bounds(h, dH, n, ldh, lo, hi));
    *emin = lo;
    *emax = hi;
    return CHEBDM_OK;
}

int chebdm_bounds_lanczos(chebdm_handle h, const double* dH, int64_t n, int64_t ldh, int32_t steps, double margin,
                          uint64_t seed, double* emin, double* emax, double* alpha_out, double* beta_out,
                          int32_t* steps_done) {
    if (!h || !emin || !emax) return fail(CHEBDM_ERR_ARG, "NULL argument");
    CHECK(validate_matrix(dH, n, ldh));
    if (steps < 1 || steps > kMaxLanczosSteps) return fail(CHEBDM_ERR_ARG, "steps must be in [1, 128]");
    if (!(margin >= 0.0) || !std::isfinite(margin)) return fail(CHEBDM_ERR_ARG, "margin must be finite and >= 0");
    CHECK(set_device(h));
    CHECK(ensure_small(h, 0));
    HIP_TRY(launch_gershgorin(dH, n, ldh, h->partial, kPartialDoubles, h->scal, h->stream));
    CHECK(lanczos_on_device(h, dH, n, ldh, steps, margin, seed));
    const int k = (int)std::min<int64_t>(steps, n);
    const LanczosWork L = lanczos_layout(h->lz, n, k);
    std::vector<double> ab(2 * (size_t)k);
    int32_t st[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(ab.data(), L.alpha, sizeof(double) * 2 * (size_t)k, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpyAsync(st, L.state, sizeof(st), hipMemcpyDeviceToHost, h->stream));
    CHECK(read_scalars(h));
    if (h->h_scal->nonfinite) return fail(CHEBDM_ERR_NONFINITE, "H holds NaN or Inf");
    *emin = h->h_scal->emin;
    *emax = h->h_scal->emax;
    const int done = st[1];
    if (alpha_out)
        for (int i = 0; i < steps; ++i) alpha_out[i] = i < done ? ab[i] : 0.0;
    if (beta_out)
        for (int i = 0; i < steps; ++i) beta_out[i] = i < done ? ab[k + i] : 0.0;
    if (steps_done) *steps_done = done;
    return CHEBDM_OK;
}

int chebdm_commutator_norm(chebdm_handle h, const double* dH, int64_t ldh, const double* dD, int64_t ldd,
                           int64_t n, double* out) {
    if (!h || !out) return fail(CHEBDM_ERR_ARG, "NULL argument");
    CHECK(validate_matrix(dH, n, ldh));
    if (!dD || ldd < n) return fail(CHEBDM_ERR_ARG, "D is NULL or ldd < n");
    CHECK(set_device(h));
    CHECK(ensure_small(h, 0));
    Plan pl;
    pl.n = n;
    pl.ld = round_up(n, 128);
    pl.elem = 8;
    CHECK(ensure_mats(h, pl, 2));
    double* w = static_cast<double*>(h->mats);
    HIP_TRY(launch_commutator(dH, ldh, dD, ldd, n, pl.ld, w, w + pl.ld * pl.ld, h->partial, h->stream));
    HIP_TRY(hipMemcpyAsync(out, h->partial, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return CHEBDM_OK;
}

int chebdm_coeffs(chebdm_handle h, double beta, double mu, double emin, double emax, int32_t order,
                  int32_t n_quad, double* c_out) {
    if (!h || !c_out) return fail(CHEBDM_ERR_ARG, "NULL argument");
    if (order < 0 || order + 1 > kSmallVec) return fail(CHEBDM_ERR_ARG, "order out of range");
    if (!(beta > 0.0) || !std::isfinite(beta) || !std::isfinite(mu)) return fail(CHEBDM_ERR_ARG, "beta must be > 0");
    if (!std::isfinite(emin) || !std::isfinite(emax) || !(emax > emin))
        return fail(CHEBDM_ERR_ARG, "need finite emin < emax");
    if (n_quad < 0) return fail(CHEBDM_ERR_ARG, "n_quad < 0");
    CHECK(set_device(h));
    Plan pl;
    pl.order = order;
    pl.M = n_quad;
    CHECK(plan_quadrature(pl, beta, emin, emax));
    CHECK(ensure_small(h, pl.M));
    HIP_TRY(launch_set_scalars(h->scal, emin, emax, beta, mu, 1, 0.0, 0.0, 0, h->stream));
    HIP_TRY(launch_fermi_coeffs(order, pl.M, h->scal, h->ftab, h->c, h->stream, pl.damping));
    HIP_TRY(hipMemcpyAsync(c_out, h->c, sizeof(double) * (size_t)(order + 1), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return CHEBDM_OK;
}

int chebdm_block_coeffs(chebdm_handle h, const double* c, int32_t order, int32_t giant_form, int32_t k_override,
                        int32_t* k_out, int32_t* m_out, double* coef_out) {
    if (!h || !k_out || !m_out) return fail(CHEBDM_ERR_ARG, "NULL argument");
    if (order < 0) return fail(CHEBDM_ERR_ARG, "order < 0");
    if (giant_form != CHEBDM_GIANT_COMPOSITION && giant_form != CHEBDM_GIANT_POWER)
        return fail(CHEBDM_ERR_ARG, "unknown giant-step form");
    if (k_override < 0) return fail(CHEBDM_ERR_ARG, "k_override < 0");
    Plan pl;
    pl.order = order;
    pl.k = k_override;
    CHECK(plan_split(pl));
    *k_out = pl.k;
    *m_out = pl.m;
    if (!coef_out) return CHEBDM_OK;
    if (!c) return fail(CHEBDM_ERR_ARG, "c is NULL");
    CHECK(set_device(h));
    CHECK(ensure_small(h, 0));
    HIP_TRY(hipMemcpyAsync(h->c, c, sizeof(double) * (size_t)(order + 1), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(launch_block_coeffs(h->c, order, pl.k, pl.m, giant_form, h->coef, h->stream));
    HIP_TRY(hipMemcpyAsync(coef_out, h->coef, sizeof(double) * (size_t)pl.k * pl.m, hipMemcpyDeviceToHost,
                           h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return CHEBDM_OK;
}

int chebdm_density(chebdm_handle h, const double* dH, int64_t n, int64_t ldh, double beta, double mu,
                   int32_t order, const chebdm_opts* opts, double emin, double emax, double* dD, int64_t ldd,
                   chebdm_info* info) {
    if (!h) return fail(CHEBDM_ERR_ARG, "handle is NULL");
    CHECK(validate_matrix(dH, n, ldh));
    if (!dD || ldd < n) return fail(CHEBDM_ERR_ARG, "D is NULL or ldd < n");
    if (order < 0) return fail(CHEBDM_ERR_ARG, "order < 0");
    if (!(beta > 0.0) || !std::isfinite(beta) || !std::isfinite(mu)) return fail(CHEBDM_ERR_ARG, "beta must be > 0");
    const bool bounds_dev = std::isnan(emin) || std::isnan(emax);   // Gershgorin bounds land in the scalars
    Plan pl;
    pl.n = n;
    pl.order = order;
    CHECK(check_opts(opts, pl));
    CHECK(plan_split(pl));
    CHECK(set_device(h));
    CHECK(resolve_bounds(h, dH, n, ldh, emin, emax, &pl));
    CHECK(ensure_small(h, 0));
    if (emax == emin) {
        // H = cI: D = f(c) I exactly (no spectrum map exists)
        const double occ = fermi_energy(emin, beta, mu);
        HIP_TRY(launch_fill_identity(dD, n, ldd, occ, h->stream));
        if (info) {
            HIP_TRY(hipStreamSynchronize(h->stream));
            pl.M = 0;
            fill_info(info, pl, emin, emax, mu, occ * (double)n, 0.0, 0, CHEBDM_OK);
        }
        return CHEBDM_OK;
    }
    CHECK(plan_quadrature(pl, beta, emin, emax));
    CHECK(ensure_small(h, pl.M));
    pl.ld = round_up(n, 128);
    CHECK(ensure_mats(h, pl, pl.k + pl.m));
    const std::vector<char> key = replay_key(2, pl, h, dH, ldh, dD, ldd, beta, mu, bounds_dev, emin, emax);
    CHECK(run_replayed(h, 2, key, &pl.n_gemm, [&]() -> int {
        pl.n_gemm = 0;
        HIP_TRY(launch_set_scalars(h->scal, emin, emax, beta, mu, 1, 0.0, pl.tol, pl.max_iter, h->stream,
                                   bounds_dev));
        HIP_TRY(launch_shift(dH, n, ldh, h->scal, tslot(h, pl, 1), pl.ld, pl.prec, h->stream));
        HIP_TRY(launch_fermi_coeffs(order, pl.M, h->scal, h->ftab, h->c, h->stream, pl.damping));
        HIP_TRY(launch_block_coeffs(h->c, order, pl.k, pl.m, pl.form, h->coef, h->stream));
        CHECK(baby_steps(h, pl, &pl.n_gemm));
        CHECK(giant_steps(h, pl, dD, ldd, &pl.n_gemm));
        return 0;
    }));
    if (info) {
        CHECK(read_scalars(h));
        fill_info(info, pl, emin, emax, mu, *h->h_trD, 0.0, 0, CHEBDM_OK);
    }
    return CHEBDM_OK;
}

int chebdm_mu_search(chebdm_handle h, const double* dH, int64_t n, int64_t ldh, double beta, double n_elec,
                     int32_t order, const chebdm_opts* opts, double emin, double emax, double* mu_out, double* dD,
                     int64_t ldd, chebdm_info* info) {
    if (!h || !mu_out) return fail(CHEBDM_ERR_ARG, "NULL argument");
    CHECK(validate_matrix(dH, n, ldh));
    if (dD && ldd < n) return fail(CHEBDM_ERR_ARG, "ldd < n");
    if (order < 0) return fail(CHEBDM_ERR_ARG, "order < 0");
    if (!(beta > 0.0) || !std::isfinite(beta)) return fail(CHEBDM_ERR_ARG, "beta must be > 0");
    if (!(n_elec > 0.0) || !(n_elec < (double)n)) return fail(CHEBDM_ERR_ARG, "need 0 < n_elec < n");
    const bool bounds_dev = std::isnan(emin) || std::isnan(emax);   // Gershgorin bounds land in the scalars
    Plan pl;
    pl.n = n;
    pl.order = order;
    CHECK(check_opts(opts, pl));
    CHECK(plan_split(pl));
    CHECK(set_device(h));
    CHECK(resolve_bounds(h, dH, n, ldh, emin, emax, &pl));
    CHECK(ensure_small(h, 0));
    if (emax == emin) {
        // H = cI: tr f(c) I = n_elec fixes the occupation n_elec/n and mu in closed form
        const double occ = n_elec / (double)n;
        const double mu = emin - std::log(1.0 / occ - 1.0) / beta;
        *mu_out = mu;
        if (dD) HIP_TRY(launch_fill_identity(dD, n, ldd, occ, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        fill_info(info, pl, emin, emax, mu, n_elec, 0.0, 0, CHEBDM_OK);
        return CHEBDM_OK;
    }
    CHECK(plan_quadrature(pl, beta, emin, emax));
    CHECK(ensure_small(h, pl.M));
    pl.ld = round_up(n, 128);
    pl.split_h = two_chain_split(pl, dD != nullptr);
    pl.split_q = four_chain_split(pl, pl.split_h);
    CHECK(ensure_mats(h, pl, pl.k + pl.m + extra_chain_slots(pl)));
    const int slot = dD ? 0 : 1;
    const std::vector<char> key = replay_key(slot, pl, h, dH, ldh, dD, dD ? ldd : 0, beta, n_elec, bounds_dev,
                                             emin, emax);
    CHECK(run_replayed(h, slot, key, &pl.n_gemm, [&]() -> int {
        pl.n_gemm = 0;
        HIP_TRY(launch_set_scalars(h->scal, emin, emax, beta, 0.0, 0, n_elec, pl.tol, pl.max_iter, h->stream,
                                   bounds_dev));
        HIP_TRY(launch_shift(dH, n, ldh, h->scal, tslot(h, pl, 1), pl.ld, pl.prec, h->stream));
        CHECK(baby_steps(h, pl, &pl.n_gemm));
        CHECK(moments_on_device(h, pl, &pl.n_gemm));
        size_t ev = (size_t)-1;
        if (h->prof) CHECK(prof_begin(h, PROF_SEARCH, 0, 0.0, 0.0, &ev));
        HIP_TRY(launch_dct3(h->tau, order, pl.M, h->w, h->xtab, h->stream, pl.damping));
        HIP_TRY(launch_bisect(h->w, h->xtab, pl.M, h->scal, pl.search, h->ftab, h->stream));
        if (h->prof) CHECK(prof_end(h, ev));
        if (dD) {
            HIP_TRY(launch_fermi_coeffs(order, pl.M, h->scal, h->ftab, h->c, h->stream, pl.damping));
            HIP_TRY(launch_block_coeffs(h->c, order, pl.k, pl.m, pl.form, h->coef, h->stream));
            if (pl.split_h > 0) HIP_TRY(launch_split_blocks(h->coef, pl.k, pl.m, pl.split_h, h->stream));
            if (pl.split_q > 0) {
                HIP_TRY(launch_split_blocks(h->coef, pl.k, pl.split_h, pl.split_q, h->stream));
                HIP_TRY(launch_split_blocks(h->coef + (int64_t)pl.split_h * pl.k, pl.k, pl.m - pl.split_h,
                                            pl.split_q, h->stream));
            }
            CHECK(giant_steps(h, pl, dD, ldd, &pl.n_gemm));
        }
        return 0;
    }));
    CHECK(read_scalars(h));
    const DevScalars& s = *h->h_scal;
    const double mu = s.cen + s.half * s.mu_s;
    *mu_out = mu;
    const int status = s.status;
    const double tr = dD ? *h->h_trD : s.trace;
    fill_info(info, pl, emin, emax, mu, tr, std::fabs(s.trace - n_elec), s.iters, status);
    if (status == CHEBDM_ERR_BRACKET)
        return fail(CHEBDM_ERR_BRACKET, "n_elec is not inside (t(mu~=-1), t(mu~=1)) of the expansion");
    return status;
}

int chebdm_workspace_size(chebdm_handle h, int64_t n, int32_t order, const chebdm_opts* opts, size_t* bytes) {
    (void)h;
    if (!bytes) return fail(CHEBDM_ERR_ARG, "NULL argument");
    if (n < 1) return fail(CHEBDM_ERR_ARG, "n < 1");
    if (order < 0) return fail(CHEBDM_ERR_ARG, "order < 0");
    Plan pl;
    pl.n = n;
    pl.order = order;
    CHECK(check_opts(opts, pl));
    CHECK(plan_split(pl));
    const int64_t ld = round_up(n, 128);
    const int64_t M = opts && opts->n_quad > 0 ? opts->n_quad : (int64_t)1 << 16;
    const bool comp = pl.form == CHEBDM_GIANT_COMPOSITION && pl.chains != 1;
    const bool four = comp && pl.m >= 8 && (pl.chains == 4 || (pl.chains == 0 && four_chains_pay(pl)));
    const int64_t slots = pl.k + pl.m + (comp && pl.m >= 4 ? 1 : 0) + (four ? 1 : 0);
    *bytes = (size_t)slots * (size_t)ld * (size_t)ld * pl.elem + small_bytes_for(M);
    *bytes += kGemmScratchBytes;
    return CHEBDM_OK;
}

int chebdm_moments(chebdm_handle h, const double* dH, int64_t n, int64_t ldh, int32_t order,
                   const chebdm_opts* opts, double emin, double emax, double* tau_out) {
    if (!h || !tau_out) return fail(CHEBDM_ERR_ARG, "NULL argument");
    CHECK(validate_matrix(dH, n, ldh));
    if (order < 0) return fail(CHEBDM_ERR_ARG, "order < 0");
    Plan pl;
    pl.n = n;
    pl.order = order;
    CHECK(check_opts(opts, pl));
    CHECK(plan_split(pl));
    CHECK(set_device(h));
    CHECK(resolve_bounds(h, dH, n, ldh, emin, emax, &pl));
    if (!(emax > emin)) return fail(CHEBDM_ERR_ARG, "moments need emin < emax");
    CHECK(ensure_small(h, 0));
    pl.ld = round_up(n, 128);
    CHECK(ensure_mats(h, pl, pl.k + pl.m));
    HIP_TRY(launch_set_scalars(h->scal, emin, emax, 1.0, 0.0, 0, 0.0, pl.tol, pl.max_iter, h->stream));
    HIP_TRY(launch_shift(dH, n, ldh, h->scal, tslot(h, pl, 1), pl.ld, pl.prec, h->stream));
    CHECK(baby_steps(h, pl, &pl.n_gemm));
    CHECK(moments_on_device(h, pl, &pl.n_gemm));
    HIP_TRY(hipMemcpyAsync(tau_out, h->tau, sizeof(double) * (size_t)(order + 1), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return CHEBDM_OK;
}

}  // extern "C"

extern "C" {

int chebdm_profile_enable(chebdm_handle h, int enable) {
    if (!h) return fail(CHEBDM_ERR_ARG, "handle is NULL");
    CHECK(set_device(h));
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->prof = enable != 0;
    h->ev_used = 0;
    return CHEBDM_OK;
}

int chebdm_profile_read(chebdm_handle h, chebdm_profile* out) {
    if (!h || !out) return fail(CHEBDM_ERR_ARG, "NULL argument");
    CHECK(set_device(h));
    HIP_TRY(hipStreamSynchronize(h->stream));
    std::memset(out, 0, sizeof(*out));
    for (size_t i = 0; i < h->ev_used; ++i) {
        const chebdm_ctx::Ev& e = h->ev[i];
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, e.a, e.b));
        if (e.kind == PROF_GEMM) {
            out->gemm_launches += 1;
            out->gemm_products += e.products;
            out->gemm_ms += ms;
            out->gemm_flop += e.flop;
        } else if (e.kind == PROF_COMBINE) {
            out->combine_calls += 1;
            out->combine_ms += ms;
            out->combine_bytes += e.bytes;
        } else if (e.kind == PROF_GRAM) {
            out->gram_calls += 1;
            out->gram_ms += ms;
            out->gram_bytes += e.bytes;
        } else {
            out->search_calls += 1;
            out->search_ms += ms;
        }
    }
    h->ev_used = 0;
    return CHEBDM_OK;
}

}  // extern "C"
