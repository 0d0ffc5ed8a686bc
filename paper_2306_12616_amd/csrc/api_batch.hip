// Batched path host side: a plan for many Hamiltonians of different n with a
// common order, run as one HIP graph (captured on first use, replayed after).
//
// Per problem the device runs the same hot path as chebdm_mu_search:
// Gershgorin bounds (then Lanczos bounds inside them, if asked), H~, sequential baby steps T_2..T_k, ladder T_{2k}..,
// Gram moments, DCT-III + bisection, coefficients at the found mu, block
// sums, Clenshaw giant steps into the caller's D.  Every product step of all
// problems is one persistent launch over a shared list of (problem, tile)
// items; the tuner picks each size bucket's tile edge and the item order by
// timing candidates on the plan's own workspace.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "cheb_dev.h"
#include "ctx.h"
#include "internal.h"

using namespace chebdm;

namespace {

constexpr int kGramBlocks = 16;     // Gram partial blocks per problem
constexpr int kBuckets = 4;         // tuning buckets of n: <=256, <=512, <=768, larger
constexpr int64_t kDefaultQuadCap = 65536;

int bucket_of(int64_t n) { return n <= 256 ? 0 : (n <= 512 ? 1 : (n <= 768 ? 2 : 3)); }

}  // namespace

struct chebdm_batch_ctx {
    chebdm_handle h = nullptr;
    hipStream_t bs = nullptr;      // own stream: graphs cannot be captured on the legacy stream
    hipEvent_t ready = nullptr;
    BatchDims d{};
    double tol = 1e-10;
    int max_iter = 200;
    size_t elem = 8;
    int steps_pre = 0, steps = 0;  // product steps before the moments, all product steps
    std::vector<int64_t> n, ld, off;
    // schedule (tuner)
    int tile_of_bucket[kBuckets] = {64, 64, 64, 64};
    int order_mode = 0;            // 0: problems by decreasing n, 1: problems in input order
    bool tuned = false;
    std::string report;
    int grid = 1024;
    int nitems = 0;
    // device memory
    void* mats = nullptr;
    size_t mats_bytes = 0;
    void* dev = nullptr;           // all small device buffers
    BatchGeom* geo = nullptr;
    BatchProblem* tab = nullptr;
    TileItem* items = nullptr;
    void* descs = nullptr;         // [steps][count] GemmDesc<T>
    int* counters = nullptr;
    DevScalars* scal = nullptr;
    int64_t* mq = nullptr;
    double *colsum = nullptr, *trb = nullptr, *partial = nullptr, *gram = nullptr, *tau = nullptr;
    double *w = nullptr, *x = nullptr, *ftab = nullptr, *c = nullptr, *coef = nullptr, *mu = nullptr, *trD = nullptr;
    // pinned host mirrors
    void* host = nullptr;
    BatchProblem* h_tab = nullptr;
    DevScalars* h_scal = nullptr;
    double *h_mu = nullptr, *h_trD = nullptr;
    // chemical-potential search: 0 bisection, 1 safeguarded Newton, 2 network guess + Newton
    int search_mode = 0;
    const float* mlp_w = nullptr;
    double mlp_delta = 0.02;
    float *feat = nullptr, *mu_hat = nullptr, *mlp_work = nullptr;
    // Lanczos bounds (opts.bounds): per-problem workspace, steps and margin; lz == nullptr: Gershgorin
    double* lz = nullptr;
    int64_t lz_stride = 0;
    int lz_steps = 0;
    double lz_margin = 0.01;
    // graphs: [0] with the density, [1] moments and mu only
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    bool have_run = false;
};

namespace {

size_t desc_size(const chebdm_batch_ctx* b) { return b->elem == 8 ? sizeof(GemmDesc<double>) : sizeof(GemmDesc<float>); }

void* slot_ptr(chebdm_batch_ctx* b, int p, int64_t s) {
    return static_cast<char*>(b->mats) + (size_t)(b->off[p] + s * b->ld[p] * b->ld[p]) * b->elem;
}

void drop_graph(chebdm_batch_ctx* b) {
    for (int i = 0; i < 2; ++i) {
        if (b->exec[i]) (void)hipGraphExecDestroy(b->exec[i]);
        if (b->graph[i]) (void)hipGraphDestroy(b->graph[i]);
        b->exec[i] = nullptr;
        b->graph[i] = nullptr;
    }
}

// Geometry (tile edges) and the shared item list for the current schedule.
int upload_schedule(chebdm_batch_ctx* b) {
    const int count = b->d.count;
    std::vector<BatchGeom> geo(count);
    std::vector<int64_t> colsum_off(count);
    int64_t acc = 0;
    for (int p = 0; p < count; ++p) {
        colsum_off[p] = acc;
        acc += b->n[p];
    }
    for (int p = 0; p < count; ++p) {
        int tile = b->tile_of_bucket[bucket_of(b->n[p])];
        // a 48-tile grid must stay inside the workspace matrix (ld = round_up(n, 128))
        if (tile == 48 && (b->n[p] + 47) / 48 * 48 > b->ld[p]) tile = 64;
        geo[p] = BatchGeom{b->n[p], b->ld[p], b->off[p], colsum_off[p], tile, (int32_t)((b->n[p] + tile - 1) / tile)};
    }
    std::vector<int> order(count);
    for (int p = 0; p < count; ++p) order[p] = p;
    if (b->order_mode == 0)
        std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return b->n[a] > b->n[c]; });
    std::vector<TileItem> items;
    for (int p : order) {
        const int nt = geo[p].ntile;
        for (int t = 0; t < nt * (nt + 1) / 2; ++t) items.push_back(TileItem{p, t});
    }
    if (items.size() > (size_t)0x7fffffff) return fail(CHEBDM_ERR_ARG, "too many tiles in the batch");
    b->nitems = (int)items.size();
    if (b->items) HIP_TRY(hipFree(b->items));
    b->items = nullptr;
    HIP_TRY(hipMalloc(&b->items, sizeof(TileItem) * items.size()));
    HIP_TRY(hipMemcpy(b->items, items.data(), sizeof(TileItem) * items.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(b->geo, geo.data(), sizeof(BatchGeom) * count, hipMemcpyHostToDevice));
    drop_graph(b);
    return 0;
}

template <typename T>
void fill_descs(chebdm_batch_ctx* b, std::vector<GemmDesc<T>>& v) {
    const int count = b->d.count, k = b->d.k, m = b->d.m, lmax = b->d.lmax;
    v.assign((size_t)b->steps * count, GemmDesc<T>{});
    auto S = [&](int p, int64_t s) { return (T*)slot_ptr(b, p, s); };
    auto lslot = [&](int l) -> int64_t { return l == 1 ? k - 1 : k + l - 2; };
    for (int p = 0; p < count; ++p) {
        int s = 0;
        // baby steps: T_{i+1} = 2 T_1 T_i - T_{i-1}, T_0 = I (slot i-1 holds T_i)
        for (int i = 1; i < k; ++i, ++s)
            v[(size_t)s * count + p] = GemmDesc<T>{S(p, 0), S(p, i - 1), i == 1 ? nullptr : S(p, i - 2), nullptr,
                                                   S(p, i), b->ld[p], 2.0, -1.0, 0.0, i == 1 ? -1.0 : 0.0, 0, 0};
        // ladder: T_{(l+1)k} = 2 T_k T_{lk} - T_{(l-1)k}
        for (int l = 1; l + 1 <= lmax; ++l, ++s)
            v[(size_t)s * count + p] =
                GemmDesc<T>{S(p, k - 1), S(p, lslot(l)), l == 1 ? nullptr : S(p, lslot(l - 1)), nullptr,
                            S(p, lslot(l + 1)), b->ld[p], 2.0, -1.0, 0.0, l == 1 ? -1.0 : 0.0, 0, 0};
        // Clenshaw over T_k blocks: B_l = R_l + 2 Y B_{l+1} - B_{l+2} (in place), D = R_0 + Y B_1 - B_2
        auto R = [&](int l) { return S(p, k + l); };
        for (int l = m - 2; l >= 1; --l, ++s)
            v[(size_t)s * count + p] = GemmDesc<T>{S(p, k - 1), R(l + 1), (l + 2 <= m - 1) ? R(l + 2) : nullptr,
                                                   R(l), R(l), b->ld[p], 2.0, -1.0, 1.0, 0.0, 0, 0};
        v[(size_t)s * count + p] = GemmDesc<T>{S(p, k - 1), R(1), m >= 3 ? R(2) : nullptr, R(0), nullptr, 0,
                                               1.0, -1.0, 1.0, 0.0, 1, 0};   // Out/ld_out patched per run
    }
}

int upload_descs(chebdm_batch_ctx* b) {
    if (b->elem == 8) {
        std::vector<GemmDesc<double>> v;
        fill_descs<double>(b, v);
        HIP_TRY(hipMemcpy(b->descs, v.data(), sizeof(GemmDesc<double>) * v.size(), hipMemcpyHostToDevice));
    } else {
        std::vector<GemmDesc<float>> v;
        fill_descs<float>(b, v);
        HIP_TRY(hipMemcpy(b->descs, v.data(), sizeof(GemmDesc<float>) * v.size(), hipMemcpyHostToDevice));
    }
    return 0;
}

const void* step_descs(const chebdm_batch_ctx* b, int s) {
    return static_cast<const char*>(b->descs) + (size_t)s * b->d.count * desc_size(b);
}

int gemm_step(chebdm_batch_ctx* b, int s, hipStream_t st, bool prof) {
    size_t ev = (size_t)-1;
    if (prof) {
        double flop = 0.0;
        for (int p = 0; p < b->d.count; ++p) flop += sym_product_flop(b->n[p]);
        CHECK(prof_begin(b->h, PROF_GEMM, b->d.count, flop, 0.0, &ev));
    }
    HIP_TRY(launch_batch_gemm(b->d.prec, step_descs(b, s), b->geo, b->items, b->nitems, b->counters + s, b->grid, st));
    if (prof) CHECK(prof_end(b->h, ev));
    return 0;
}

// The whole batched hot path, enqueued on st (captured into the graph, or run
// eagerly with launch timing when the handle's profiling is on).
int enqueue(chebdm_batch_ctx* b, hipStream_t st, bool prof, bool with_density) {
    const BatchDims& d = b->d;
    HIP_TRY(launch_batch_zero(b->counters, b->steps, st));
    if (with_density) HIP_TRY(launch_batch_patch(d, b->tab, const_cast<void*>(step_descs(b, b->steps - 1)), st));
    HIP_TRY(launch_batch_bounds(d, b->tab, b->geo, b->colsum, b->scal, st));
    if (b->lz) {
        LanczosRun r{};
        r.tab = b->tab;
        r.geo = b->geo;
        r.s = b->scal;
        r.base = b->lz;
        r.stride = b->lz_stride;
        r.nmax = d.nmax;
        r.steps = b->lz_steps;
        r.margin = b->lz_margin;
        r.seed = 0;
        HIP_TRY(launch_lanczos_run(r, d.count, st));
    }
    HIP_TRY(launch_batch_setup(d, b->tab, b->geo, b->scal, b->mq, b->tol, b->max_iter, st));
    HIP_TRY(launch_batch_shift(d, b->tab, b->geo, b->scal, b->mats, st));
    for (int s = 0; s < b->steps_pre; ++s) CHECK(gemm_step(b, s, st, prof));
    size_t ev = (size_t)-1;
    if (prof) {
        double bytes = 0.0;
        for (int p = 0; p < d.count; ++p) bytes += (double)(d.lmax + d.k) * b->n[p] * b->n[p] * b->elem;
        CHECK(prof_begin(b->h, PROF_GRAM, 0, 0.0, bytes, &ev));
    }
    HIP_TRY(launch_batch_moments(d, b->geo, b->mats, b->trb, b->partial, kGramBlocks, b->gram, b->tau, st));
    if (prof) CHECK(prof_end(b->h, ev));
    if (prof) CHECK(prof_begin(b->h, PROF_SEARCH, 0, 0.0, 0.0, &ev));
    if (b->search_mode == 2) {
        HIP_TRY(launch_batch_features(d, b->geo, b->tau, b->scal, b->feat, st));
        HIP_TRY(launch_mlp_forward(b->mlp_w, b->feat, d.count, b->mu_hat, b->mlp_work, st));
    }
    HIP_TRY(launch_batch_search(d, b->tau, b->mq, b->w, b->x, b->scal, b->search_mode, b->mu_hat, b->mlp_delta,
                                b->ftab, st));
    if (prof) CHECK(prof_end(b->h, ev));
    if (!with_density) {
        HIP_TRY(launch_batch_finish(d, b->tab, b->geo, b->scal, b->mu, b->trD, 0, st));
        return 0;
    }
    HIP_TRY(launch_batch_coeffs(d, b->mq, b->scal, b->ftab, b->c, b->coef, st));
    if (prof) {
        double bytes = 0.0;
        for (int p = 0; p < d.count; ++p) bytes += (double)(d.k - 1 + d.m) * b->n[p] * b->n[p] * b->elem;
        CHECK(prof_begin(b->h, PROF_COMBINE, 0, 0.0, bytes, &ev));
    }
    HIP_TRY(launch_batch_combine(d, b->geo, b->coef, b->mats, st));
    if (prof) CHECK(prof_end(b->h, ev));
    for (int s = b->steps_pre; s < b->steps; ++s) CHECK(gemm_step(b, s, st, prof));
    HIP_TRY(launch_batch_finish(d, b->tab, b->geo, b->scal, b->mu, b->trD, 1, st));
    return 0;
}

// Mean time of product step 0 (T_2 = 2 T_1 T_1 - I for all problems) under the current schedule.
int time_step0(chebdm_batch_ctx* b, float* ms_out) {
    CHECK(upload_schedule(b));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(launch_batch_zero(b->counters, 1, b->bs));
    HIP_TRY(launch_batch_gemm(b->d.prec, step_descs(b, 0), b->geo, b->items, b->nitems, b->counters, b->grid, b->bs));
    const int reps = 3;
    HIP_TRY(hipEventRecord(e0, b->bs));
    for (int r = 0; r < reps; ++r) {
        HIP_TRY(launch_batch_zero(b->counters, 1, b->bs));
        HIP_TRY(launch_batch_gemm(b->d.prec, step_descs(b, 0), b->geo, b->items, b->nitems, b->counters, b->grid,
                                  b->bs));
    }
    HIP_TRY(hipEventRecord(e1, b->bs));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms_out = ms / reps;
    return 0;
}

std::string tune_key(const chebdm_batch_ctx* b) {
    int hist[kBuckets] = {0, 0, 0, 0};
    for (int64_t v : b->n) hist[bucket_of(v)]++;
    std::ostringstream os;
    os << "prec" << b->d.prec << "_order" << b->d.order << "_count" << b->d.count << "_hist" << hist[0] << "-"
       << hist[1] << "-" << hist[2] << "-" << hist[3] << "_nmax" << b->d.nmax;
    return os.str();
}

std::string tune_value(const chebdm_batch_ctx* b) {
    std::ostringstream os;
    os << "tiles=" << b->tile_of_bucket[0] << "," << b->tile_of_bucket[1] << "," << b->tile_of_bucket[2] << ","
       << b->tile_of_bucket[3] << " order=" << b->order_mode;
    return os.str();
}

bool parse_value(const std::string& v, int tiles[kBuckets], int* order) {
    int t0, t1, t2, t3, o;
    if (std::sscanf(v.c_str(), "tiles=%d,%d,%d,%d order=%d", &t0, &t1, &t2, &t3, &o) != 5) return false;
    for (int t : {t0, t1, t2, t3})
        if (t != 32 && t != 48 && t != 64) return false;
    if (o != 0 && o != 1) return false;
    tiles[0] = t0, tiles[1] = t1, tiles[2] = t2, tiles[3] = t3;
    *order = o;
    return true;
}

}  // namespace

// =================================================================== C ABI

extern "C" {

int chebdm_batch_create(chebdm_handle h, int32_t count, const int64_t* n, int32_t order, const chebdm_opts* opts,
                        int64_t max_quad, chebdm_batch* out) {
    if (!h || !n || !out) return fail(CHEBDM_ERR_ARG, "NULL argument");
    *out = nullptr;
    if (count < 1 || count > 65535) return fail(CHEBDM_ERR_ARG, "count must be in [1, 65535]");
    chebdm_opts o;
    chebdm_default_opts(&o);
    if (opts) o = *opts;
    if (o.prec < CHEBDM_FP64 || o.prec > CHEBDM_BF16X6) return fail(CHEBDM_ERR_ARG, "unknown precision");
    if (o.giant_form == CHEBDM_GIANT_POWER || o.giant_form == CHEBDM_GIANT_TWO_CHAINS ||
        o.giant_form == CHEBDM_GIANT_FOUR_CHAINS)
        return fail(CHEBDM_ERR_UNSUPPORTED, "the batched path uses the composition form in one chain only");
    if (o.giant_form < CHEBDM_GIANT_COMPOSITION || o.giant_form > CHEBDM_GIANT_FOUR_CHAINS)
        return fail(CHEBDM_ERR_ARG, "unknown giant-step form");
    if (o.bounds != CHEBDM_BOUNDS_GERSHGORIN && o.bounds != CHEBDM_BOUNDS_LANCZOS)
        return fail(CHEBDM_ERR_ARG, "unknown bounds method");
    if (o.lanczos_steps < 0 || o.lanczos_steps > kMaxLanczosSteps)
        return fail(CHEBDM_ERR_ARG, "lanczos_steps must be in [0, 128]");
    if (!(o.bounds_margin >= 0.0) || !std::isfinite(o.bounds_margin))
        return fail(CHEBDM_ERR_ARG, "bounds_margin must be finite and >= 0");
    if (o.n_quad != 0) return fail(CHEBDM_ERR_UNSUPPORTED, "the batched path sizes the quadrature per problem");
    if (o.search != CHEBDM_SEARCH_BISECTION && o.search != CHEBDM_SEARCH_NEWTON)
        return fail(CHEBDM_ERR_ARG, "unknown mu search");
    if (o.damping != CHEBDM_DAMPING_NONE && o.damping != CHEBDM_DAMPING_JACKSON)
        return fail(CHEBDM_ERR_ARG, "unknown damping");
    if (order < 2) return fail(CHEBDM_ERR_ARG, "the batched path needs order >= 2");
    int64_t k = o.k_override;
    if (k <= 0) {
        k = 1;
        while (k * k < (int64_t)order + 1) ++k;
    }
    const int64_t m = ((int64_t)order + 1 + k - 1) / k;
    if (k < 2 || k > kMaxBlocks || m < 2 || m > kMaxBlocks)
        return fail(CHEBDM_ERR_ARG, "need 2 <= k, m <= 48 (order and k_override)");
    int64_t nmax = 0;
    for (int p = 0; p < count; ++p) {
        if (n[p] < 1 || n[p] > 65535) return fail(CHEBDM_ERR_ARG, "every n must be in [1, 65535]");
        nmax = std::max(nmax, n[p]);
    }
    const int64_t mcap = max_quad > 0 ? max_quad : kDefaultQuadCap;
    if (mcap < order + 1 || mcap > (1 << 26)) return fail(CHEBDM_ERR_ARG, "max_quad out of range");
    HIP_TRY(hipSetDevice(h->device));

    chebdm_batch_ctx* b = new (std::nothrow) chebdm_batch_ctx();
    if (!b) return fail(CHEBDM_ERR_OOM, "cannot allocate the batch plan");
    b->h = h;
    b->elem = o.prec == CHEBDM_FP64 ? 8 : 4;
    b->tol = o.tol > 0.0 ? o.tol : 1e-10;
    b->max_iter = o.max_iter > 0 ? o.max_iter : 200;
    b->search_mode = o.search;
    int lmax = (order - 1) / (int)k;
    if (lmax > (int)m - 1) lmax = (int)m - 1;
    b->d = BatchDims{count, order, (int)k, (int)m, lmax, nmax, 0, mcap, o.prec, o.damping};
    b->steps_pre = (int)(k - 1) + (lmax >= 2 ? lmax - 1 : 0);
    b->steps = b->steps_pre + (int)(m - 1);
    b->n.assign(n, n + count);
    b->ld.resize(count);
    b->off.resize(count);
    int64_t tot = 0, ldmax = 0;
    for (int p = 0; p < count; ++p) {
        b->ld[p] = (n[p] + 127) / 128 * 128;
        ldmax = std::max(ldmax, b->ld[p]);
        b->off[p] = tot;
        tot += (k + m) * b->ld[p] * b->ld[p];
    }
    b->d.ldmax = ldmax;
    auto bail = [&](int rc) {
        chebdm_batch_destroy(b);
        return rc;
    };
    if (hipStreamCreateWithFlags(&b->bs, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ready, hipEventDisableTiming) != hipSuccess)
        return bail(fail(CHEBDM_ERR_HIP, "cannot create the batch stream"));
    if (o.bounds == CHEBDM_BOUNDS_LANCZOS) {
        b->lz_steps = o.lanczos_steps ? o.lanczos_steps : 40;
        b->lz_margin = o.bounds_margin > 0.0 ? o.bounds_margin : 0.01;
        b->lz_stride = (lanczos_work_doubles(nmax, b->lz_steps) + 31) / 32 * 32;
        const size_t lz_bytes = sizeof(double) * (size_t)b->lz_stride * (size_t)count;
        if (hipMalloc(&b->lz, lz_bytes) != hipSuccess) {
            b->lz = nullptr;
            (void)hipGetLastError();
            return bail(fail(CHEBDM_ERR_OOM, "cannot allocate " + std::to_string(lz_bytes) + " bytes of Lanczos workspace"));
        }
    }
    b->mats_bytes = (size_t)tot * b->elem;
    if (hipMalloc(&b->mats, b->mats_bytes) != hipSuccess) {
        b->mats = nullptr;
        (void)hipGetLastError();
        return bail(fail(CHEBDM_ERR_OOM, "cannot allocate " + std::to_string(b->mats_bytes) + " bytes of batch workspace"));
    }
    // small buffers in one allocation
    const size_t L1 = (size_t)order + 1, K = (size_t)k, M = (size_t)m, C = (size_t)count;
    int64_t ncols = 0;
    for (int64_t v : b->n) ncols += v;
    size_t bytes = 0;
    auto take = [&](size_t nb) {
        const size_t at = bytes;
        bytes += (nb + 255) / 256 * 256;
        return at;
    };
    const size_t o_geo = take(sizeof(BatchGeom) * C), o_tab = take(sizeof(BatchProblem) * C);
    const size_t o_desc = take(desc_size(b) * C * b->steps), o_cnt = take(sizeof(int) * b->steps);
    const size_t o_scal = take(sizeof(DevScalars) * C), o_mq = take(sizeof(int64_t) * C);
    const size_t o_col = take(sizeof(double) * ncols), o_trb = take(sizeof(double) * C * K);
    const size_t o_part = take(sizeof(double) * C * kGramBlocks * 48 * 48), o_gram = take(sizeof(double) * C * 48 * 48);
    const size_t o_tau = take(sizeof(double) * C * L1), o_w = take(sizeof(double) * C * mcap);
    const size_t o_x = take(sizeof(double) * C * mcap), o_f = take(sizeof(double) * C * mcap);
    const size_t o_c = take(sizeof(double) * C * L1), o_coef = take(sizeof(double) * C * K * M);
    const size_t o_mu = take(sizeof(double) * C), o_trd = take(sizeof(double) * C);
    const size_t o_feat = take(sizeof(float) * C * 64), o_muh = take(sizeof(float) * C);
    const size_t o_mlpw = take(sizeof(float) * C * 512);
    if (hipMalloc(&b->dev, bytes) != hipSuccess) {
        b->dev = nullptr;
        (void)hipGetLastError();
        return bail(fail(CHEBDM_ERR_OOM, "cannot allocate " + std::to_string(bytes) + " bytes of batch tables"));
    }
    char* base = static_cast<char*>(b->dev);
    b->geo = (BatchGeom*)(base + o_geo);
    b->tab = (BatchProblem*)(base + o_tab);
    b->descs = base + o_desc;
    b->counters = (int*)(base + o_cnt);
    b->scal = (DevScalars*)(base + o_scal);
    b->mq = (int64_t*)(base + o_mq);
    b->colsum = (double*)(base + o_col);
    b->trb = (double*)(base + o_trb);
    b->partial = (double*)(base + o_part);
    b->gram = (double*)(base + o_gram);
    b->tau = (double*)(base + o_tau);
    b->w = (double*)(base + o_w);
    b->x = (double*)(base + o_x);
    b->ftab = (double*)(base + o_f);
    b->c = (double*)(base + o_c);
    b->coef = (double*)(base + o_coef);
    b->mu = (double*)(base + o_mu);
    b->trD = (double*)(base + o_trd);
    b->feat = (float*)(base + o_feat);
    b->mu_hat = (float*)(base + o_muh);
    b->mlp_work = (float*)(base + o_mlpw);
    const size_t hbytes = sizeof(BatchProblem) * C + sizeof(DevScalars) * C + 2 * sizeof(double) * C + 256;
    if (hipHostMalloc(&b->host, hbytes, hipHostMallocDefault) != hipSuccess) {
        b->host = nullptr;
        return bail(fail(CHEBDM_ERR_OOM, "cannot allocate pinned host tables"));
    }
    char* hb = static_cast<char*>(b->host);
    b->h_tab = (BatchProblem*)hb;
    b->h_scal = (DevScalars*)(hb + sizeof(BatchProblem) * C);
    b->h_mu = (double*)(hb + sizeof(BatchProblem) * C + sizeof(DevScalars) * C);
    b->h_trD = b->h_mu + C;
    // zero padding of every workspace matrix; kernels only ever write the n x n blocks
    if (hipMemsetAsync(b->mats, 0, b->mats_bytes, b->bs) != hipSuccess ||
        hipMemsetAsync(b->dev, 0, bytes, b->bs) != hipSuccess || hipStreamSynchronize(b->bs) != hipSuccess)
        return bail(fail(CHEBDM_ERR_HIP, "cannot clear the batch workspace"));
    b->grid = batch_gemm_grid(o.prec);
    int rc = upload_descs(b);
    if (rc < 0) return bail(rc);
    rc = upload_schedule(b);
    if (rc < 0) return bail(rc);
    *out = b;
    return CHEBDM_OK;
}

int chebdm_batch_destroy(chebdm_batch b) {
    if (!b) return CHEBDM_OK;
    if (b->h) (void)hipSetDevice(b->h->device);
    if (b->bs) (void)hipStreamSynchronize(b->bs);
    drop_graph(b);
    if (b->items) (void)hipFree(b->items);
    if (b->dev) (void)hipFree(b->dev);
    if (b->mats) (void)hipFree(b->mats);
    if (b->lz) (void)hipFree(b->lz);
    if (b->host) (void)hipHostFree(b->host);
    if (b->ready) (void)hipEventDestroy(b->ready);
    if (b->bs) (void)hipStreamDestroy(b->bs);
    delete b;
    return CHEBDM_OK;
}

int chebdm_batch_tune(chebdm_batch b, const char* cache_path, char* report, int32_t report_len) {
    if (!b) return fail(CHEBDM_ERR_ARG, "batch is NULL");
    HIP_TRY(hipSetDevice(b->h->device));
    const std::string key = tune_key(b);
    bool loaded = false;
    if (cache_path && *cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            const size_t sp = line.find(' ');
            if (sp == std::string::npos || line.substr(0, sp) != key) continue;
            int tiles[kBuckets], ord = 0;
            if (parse_value(line.substr(sp + 1), tiles, &ord)) {
                std::copy(tiles, tiles + kBuckets, b->tile_of_bucket);
                b->order_mode = ord;
                loaded = true;
            }
        }
    }
    std::ostringstream rep;
    if (loaded) {
        CHECK(upload_schedule(b));
        rep << "loaded " << key << " -> " << tune_value(b);
    } else {
        int present[kBuckets] = {0, 0, 0, 0};
        for (int64_t v : b->n) present[bucket_of(v)] = 1;
        std::fill(b->tile_of_bucket, b->tile_of_bucket + kBuckets, 64);
        b->order_mode = 0;
        float best = 0.0f;
        CHECK(time_step0(b, &best));
        rep << "base tiles=64 order=0: " << best << " ms;";
        for (int bk = 0; bk < kBuckets; ++bk) {
            if (!present[bk]) continue;
            int keep = 64;
            for (int cand : {48, 32}) {
                b->tile_of_bucket[bk] = cand;
                float t = 0.0f;
                CHECK(time_step0(b, &t));
                rep << " bucket" << bk << " tile" << cand << ": " << t << " ms;";
                if (t < 0.98f * best) {
                    best = t;
                    keep = cand;
                }
            }
            b->tile_of_bucket[bk] = keep;
        }
        b->order_mode = 1;
        float t = 0.0f;
        CHECK(time_step0(b, &t));
        rep << " order1: " << t << " ms;";
        if (t < 0.98f * best) best = t;
        else b->order_mode = 0;
        CHECK(upload_schedule(b));
        rep << " chose " << tune_value(b) << " (" << best << " ms per product step)";
        if (cache_path && *cache_path) {
            std::ofstream outf(cache_path, std::ios::app);
            if (outf) outf << key << " " << tune_value(b) << "\n";
        }
    }
    b->tuned = true;
    b->report = rep.str();
    if (report && report_len > 0) {
        std::strncpy(report, b->report.c_str(), (size_t)report_len - 1);
        report[report_len - 1] = '\0';
    }
    return CHEBDM_OK;
}

int chebdm_batch_mu_search(chebdm_batch b, const double* const* dH, const int64_t* ldh, const double* beta,
                           const double* n_elec, double* const* dD, const int64_t* ldd, double* mu_out,
                           int32_t* status_out, int32_t* iters_out, double* trace_out) {
    if (!b || !dH || !ldh || !beta || !n_elec || !mu_out || (dD && !ldd))
        return fail(CHEBDM_ERR_ARG, "NULL argument");
    chebdm_handle h = b->h;
    HIP_TRY(hipSetDevice(h->device));
    const int count = b->d.count;
    const bool with_density = dD != nullptr;
    for (int p = 0; p < count; ++p) {
        if (!dH[p] || (with_density && !dD[p])) return fail(CHEBDM_ERR_ARG, "NULL matrix in the batch");
        if (ldh[p] < b->n[p] || (with_density && ldd[p] < b->n[p]))
            return fail(CHEBDM_ERR_ARG, "leading dimension smaller than n");
        b->h_tab[p] = BatchProblem{dH[p], with_density ? dD[p] : nullptr, ldh[p], with_density ? ldd[p] : 0,
                                   beta[p], n_elec[p]};
    }
    if (b->search_mode == 2 && !b->mlp_w) return fail(CHEBDM_ERR_ARG, "network search mode without weights");
    const int gi = with_density ? 0 : 1;
    hipStream_t st;
    if (h->prof) {
        // eager run on the handle's stream with launch timing
        st = h->stream;
        HIP_TRY(hipMemcpyAsync(b->tab, b->h_tab, sizeof(BatchProblem) * count, hipMemcpyHostToDevice, st));
        CHECK(enqueue(b, st, true, with_density));
    } else {
        st = b->bs;
        if (!b->exec[gi]) {
            HIP_TRY(hipStreamBeginCapture(b->bs, hipStreamCaptureModeThreadLocal));
            const int rc = enqueue(b, b->bs, false, with_density);
            hipGraph_t g = nullptr;
            const hipError_t ec = hipStreamEndCapture(b->bs, &g);
            if (rc < 0) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            HIP_TRY(ec);
            b->graph[gi] = g;
            HIP_TRY(hipGraphInstantiate(&b->exec[gi], b->graph[gi], nullptr, nullptr, 0));
        }
        // the caller's H was written on the handle's stream
        HIP_TRY(hipEventRecord(b->ready, h->stream));
        HIP_TRY(hipStreamWaitEvent(b->bs, b->ready, 0));
        HIP_TRY(hipMemcpyAsync(b->tab, b->h_tab, sizeof(BatchProblem) * count, hipMemcpyHostToDevice, b->bs));
        HIP_TRY(hipGraphLaunch(b->exec[gi], b->bs));
    }
    HIP_TRY(hipMemcpyAsync(b->h_scal, b->scal, sizeof(DevScalars) * count, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(b->h_mu, b->mu, sizeof(double) * count, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(b->h_trD, b->trD, sizeof(double) * count, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    b->have_run = true;
    int worst = CHEBDM_OK;
    for (int p = 0; p < count; ++p) {
        const int s = b->h_scal[p].status;
        mu_out[p] = b->h_mu[p];
        if (status_out) status_out[p] = s;
        if (iters_out) iters_out[p] = b->h_scal[p].iters;
        if (trace_out) trace_out[p] = b->h_trD[p];
        if (s < 0 && (worst >= 0 || s < worst)) worst = s;
        else if (s > 0 && worst == CHEBDM_OK) worst = s;
    }
    if (worst < 0) return fail(worst, "at least one problem of the batch failed (see status_out)");
    return worst;
}

int chebdm_batch_set_search(chebdm_batch b, int32_t mode, const float* dW, double delta) {
    if (!b) return fail(CHEBDM_ERR_ARG, "batch is NULL");
    if (mode < 0 || mode > 2) return fail(CHEBDM_ERR_ARG, "unknown search mode");
    if (mode == 2 && (!dW || !(delta > 0.0) || !(delta <= 2.0)))
        return fail(CHEBDM_ERR_ARG, "the network mode needs weights and 0 < delta <= 2");
    b->search_mode = mode;
    b->mlp_w = mode == 2 ? dW : nullptr;
    b->mlp_delta = mode == 2 ? delta : 0.0;
    drop_graph(b);
    return CHEBDM_OK;
}

int chebdm_batch_stats(chebdm_batch b, int32_t* evals, int32_t* learned, double* mu_s, double* beta_s) {
    if (!b) return fail(CHEBDM_ERR_ARG, "batch is NULL");
    if (!b->have_run) return fail(CHEBDM_ERR_ARG, "no run yet");
    for (int p = 0; p < b->d.count; ++p) {
        if (evals) evals[p] = b->h_scal[p].evals;
        if (learned) learned[p] = b->h_scal[p].learned;
        if (mu_s) mu_s[p] = b->h_scal[p].mu_s;
        if (beta_s) beta_s[p] = b->h_scal[p].beta_s;
    }
    return CHEBDM_OK;
}

int chebdm_batch_features(chebdm_batch b, float* dfeat) {
    if (!b || !dfeat) return fail(CHEBDM_ERR_ARG, "NULL argument");
    if (!b->have_run) return fail(CHEBDM_ERR_ARG, "no run yet");
    HIP_TRY(hipSetDevice(b->h->device));
    HIP_TRY(launch_batch_features(b->d, b->geo, b->tau, b->scal, b->feat, b->bs));
    HIP_TRY(hipMemcpyAsync(dfeat, b->feat, sizeof(float) * 64 * (size_t)b->d.count, hipMemcpyDeviceToDevice, b->bs));
    HIP_TRY(hipStreamSynchronize(b->bs));
    return CHEBDM_OK;
}

int chebdm_batch_info(chebdm_batch b, int32_t* k, int32_t* m, int32_t* products_per_problem, int64_t* tiles_per_step,
                      double* flop_per_run) {
    if (!b) return fail(CHEBDM_ERR_ARG, "batch is NULL");
    if (k) *k = b->d.k;
    if (m) *m = b->d.m;
    if (products_per_problem) *products_per_problem = b->steps;
    if (tiles_per_step) *tiles_per_step = b->nitems;
    if (flop_per_run) {
        double f = 0.0;
        for (int64_t v : b->n) f += sym_product_flop(v);
        *flop_per_run = f * b->steps;
    }
    return CHEBDM_OK;
}

}  // extern "C"
