// Host side of the C ABI declared in include/pam.h: context, workspace,
// argument validation and orchestration of the kernels.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "pam_internal.h"

namespace pam {

static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }

pam_status ensure(pam_ctx *ctx, Buf b, size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (ctx->ws.bytes[b] >= bytes) return PAM_OK;
    if (ctx->graphs.capturing) {   // workspace is sized before a capture; the caller falls back
        set_error("workspace growth during a graph capture");
        return PAM_ERR_STATE;
    }
    if (ctx->ws.ptr[b]) {
        PAM_CHECK_HIP(hipStreamSynchronize(ctx->stream));
        PAM_CHECK_HIP(hipFree(ctx->ws.ptr[b]));
        ctx->ws.ptr[b] = nullptr;
        ctx->ws.bytes[b] = 0;
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        set_error("workspace allocation of " + std::to_string(bytes) + " bytes failed");
        return PAM_ERR_NOMEM;
    }
    ctx->ws.ptr[b] = p;
    ctx->ws.bytes[b] = bytes;
    return PAM_OK;
}

// Small host tables go through the context's pinned staging buffer.
pam_status upload_to(pam_ctx *ctx, void *dst, const void *host, size_t bytes) {
    if (bytes == 0) return PAM_OK;
    Staging &sg = ctx->staging;
    if (sg.done) PAM_CHECK_HIP(hipEventSynchronize(sg.done));
    if (sg.bytes < bytes) {
        if (sg.host) PAM_CHECK_HIP(hipHostFree(sg.host));
        sg.host = nullptr;
        sg.bytes = 0;
        PAM_CHECK_HIP(hipHostMalloc(&sg.host, bytes));
        sg.bytes = bytes;
    }
    if (!sg.done) PAM_CHECK_HIP(hipEventCreateWithFlags(&sg.done, hipEventDisableTiming));
    memcpy(sg.host, host, bytes);
    PAM_CHECK_HIP(hipMemcpyAsync(dst, sg.host, bytes, hipMemcpyHostToDevice, ctx->stream));
    PAM_CHECK_HIP(hipEventRecord(sg.done, ctx->stream));
    return PAM_OK;
}

pam_status upload(pam_ctx *ctx, Buf b, const void *host, size_t bytes) {
    pam_status st = ensure(ctx, b, bytes);
    if (st != PAM_OK) return st;
    return upload_to(ctx, ctx->ws.ptr[b], host, bytes);
}

static hipEvent_t timing_event(pam_ctx *ctx) {
    Timing &t = ctx->timing;
    if (!t.pool.empty()) {
        hipEvent_t e = t.pool.back();
        t.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

KernelTimer::KernelTimer(pam_ctx *ctx, int kind) : ctx_(ctx), kind_(kind) {
    if (!ctx_->timing.on || kind_ < 0) return;
    start_ = timing_event(ctx_);
    if (start_) (void)hipEventRecord(start_, ctx_->stream);
}

KernelTimer::~KernelTimer() {
    if (!start_) return;
    hipEvent_t stop = timing_event(ctx_);
    if (!stop) return;
    (void)hipEventRecord(stop, ctx_->stream);
    ctx_->timing.pending.push_back({kind_, {start_, stop}});
}

// refit mask (k_fit.hip)
pam_status launch_noconv_mask(pam_ctx *ctx, const pam_fit_stats *stats, int n, int32_t *mask);

// setup kernels (k_setup.hip)
pam_status launch_gather(pam_ctx *ctx, const pam_grid *g, const void *tab_dev, int n_sub,
                         int32_t n_max, const double *cell_y, const int64_t *off, double *x,
                         double *y, double *h, int32_t *cell);
pam_status launch_lattice(pam_ctx *ctx, int dim, const int32_t *g, int n_sub, int m_cap,
                          const void *tab_dev, pam_dict *dict);
size_t gather_table_bytes(int n_sub);
size_t lattice_table_bytes(int n_sub);
void build_gather_table(const pam_grid *g, void *host_tab);
void build_lattice_table(const pam_grid *g, const int32_t *gl, double sigma_factor, void *host_tab);
void axis_range(int n_cells, int n_sub, const int32_t *brk, int k, double overlap, int *first, int *last);
int64_t interface_count(int n_fields, const pam_field *fields);
// Darcy consumer (k_darcy.hip)
pam_status launch_darcy_solve(pam_ctx *ctx, const pam_darcy_opts *o, const double *k_tri,
                              double *p, int warm, int32_t *iters, double *rel_res);
pam_status launch_darcy_error(pam_ctx *ctx, const pam_darcy_opts *o, const double *p_ref,
                              const double *p, double *e_rel);
pam_status launch_darcy_coefficient(pam_ctx *ctx, const pam_darcy_opts *o, const pam_field *field,
                                    const pam_dict *dict, const double *beta, double blend,
                                    double *k_tri);
pam_status launch_darcy_cells(pam_ctx *ctx, const pam_darcy_opts *o, const double *cell_y,
                              double *k_tri);
// lambda selection (k_select.hip)
pam_status launch_cv_setup(pam_ctx *ctx, const pam_samples *S, const pam_dict *D, int K,
                           const int64_t *off_v, double *xv, double *yv, int32_t *mv, double *cv,
                           double *sv, int32_t *lv, double *beta_v, double *inv_s, int n_alpha,
                           double ratio, double rho, double *alpha, int32_t *n_failed);
pam_status launch_cv_lambda(pam_ctx *ctx, int n_sub, int K, int n_alpha, int k, double rho,
                            const double *alpha, double *l1v, double *l2v);
pam_status launch_cv_score(pam_ctx *ctx, const pam_samples *S, const pam_dict *D, int K,
                           int n_alpha, int k, const double *beta_v, const pam_fit_stats *stats_v,
                           double *score, int32_t *n_failed);
pam_status launch_cv_choose(pam_ctx *ctx, int n_sub, int n_alpha, double rho, const double *alpha,
                            const double *score, int32_t *best, double *l1, double *l2);
pam_status launch_interface_jump(pam_ctx *ctx, int n_fields, const pam_field *fields,
                                 const pam_dict *dict, const double *beta, int n, double *out);

static pam_status check_grid(const pam_grid *g, int *n_sub_total) {
    PAM_REQUIRE(g, "grid is NULL");
    PAM_REQUIRE(g->dim >= 1 && g->dim <= 3, "grid dim must be 1, 2 or 3");
    PAM_REQUIRE(g->breaks, "grid breaks are NULL");
    PAM_REQUIRE(g->overlap >= 0.0 && g->overlap < 1.0, "overlap must be in [0, 1)");
    int pos = 0, tot = 1;
    for (int a = 0; a < g->dim; ++a) {
        PAM_REQUIRE(g->n_cells[a] >= 1 && g->n_sub[a] >= 1, "cell and subdomain counts must be >= 1");
        PAM_REQUIRE(g->hi[a] > g->lo[a], "domain box must have hi > lo");
        const int32_t *b = g->breaks + pos;
        PAM_REQUIRE(b[0] == 0 && b[g->n_sub[a]] == g->n_cells[a], "breaks must span 0..n_cells");
        for (int k = 0; k < g->n_sub[a]; ++k) PAM_REQUIRE(b[k + 1] > b[k], "breaks must increase");
        pos += g->n_sub[a] + 1;
        tot *= g->n_sub[a];
    }
    *n_sub_total = tot;
    return PAM_OK;
}

// Workspace of one batched fit launch: PAM_WS_BYTES if set, else 60 % of the
// device memory free at the call, at most 160 GiB (288 GB of HBM3E per GPU:
// the 1,188 three-round layered subdomains, ~55 MB each, fit in one launch).
static size_t ws_budget() {
    const char *e = getenv("PAM_WS_BYTES");
    if (e) return (size_t)strtoull(e, nullptr, 10);
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        return (size_t)48 << 30;
    }
    return std::min<size_t>((size_t)160 << 30, free_b / 10 * 6);
}

static size_t wbytes(int prec) { return prec == PAM_PREC_F64 ? 8 : (prec == PAM_PREC_F32 ? 4 : 2); }
static size_t gbytes(int prec) { return prec == PAM_PREC_F64 ? 8 : 4; }

// ---------------------------------------------------------------- Gram tuner
// The low-precision Gram has two paths: the assembly writes the normalized
// design to HBM and the Gram tiles read it, or the row sums are taken first
// and the Gram tiles compute the design entries they need in LDS (fused: no
// design in HBM, every entry recomputed in each tile that uses it). Both give
// the same bits; which is faster depends on the tile count (M), the sample
// count (N) and the precision. The tuner times both on the first batched fit
// of a (precision, padded M, padded N) bucket and keeps the faster: in
// memory for the process and, when PAM_TUNE_CACHE names a file, as one JSON
// object per line there (read at the first lookup, appended on each new
// choice). pam_gram_path forces either path.
struct TuneEntry { int fused; double ms_materialized, ms_fused; };
static std::mutex g_tune_mu;
static std::map<std::string, TuneEntry> g_tune;
static bool g_tune_loaded = false;

static std::string tune_key(const FitArgs &a) {
    const char *pn = a.precision == PAM_PREC_F32 ? "f32" : "bf16";
    return std::string("gfx950/gram/") + pn + "/mpad" + std::to_string(a.mpad) + "/npad" + std::to_string(a.npad);
}

static void tune_load() {
    g_tune_loaded = true;
    const char *path = getenv("PAM_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char line[512];
    while (fgets(line, sizeof line, f)) {
        // {"key": "...", "path": "fused"|"materialized", "ms_materialized": x, "ms_fused": y}
        const char *k = strstr(line, "\"key\": \"");
        const char *pth = strstr(line, "\"path\": \"");
        if (!k || !pth) continue;
        k += 8;
        const char *ke = strchr(k, '"');
        if (!ke) continue;
        TuneEntry e{strncmp(pth + 9, "fused", 5) == 0 ? 1 : 0, 0.0, 0.0};
        const char *mm = strstr(line, "\"ms_materialized\": ");
        const char *mf = strstr(line, "\"ms_fused\": ");
        if (mm) e.ms_materialized = atof(mm + 19);
        if (mf) e.ms_fused = atof(mf + 12);
        g_tune[std::string(k, ke - k)] = e;
    }
    fclose(f);
}

static void tune_store(const std::string &key, const TuneEntry &e) {
    const char *path = getenv("PAM_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "{\"key\": \"%s\", \"path\": \"%s\", \"ms_materialized\": %.4f, \"ms_fused\": %.4f}\n", key.c_str(),
            e.fused ? "fused" : "materialized", e.ms_materialized, e.ms_fused);
    fclose(f);
}

// Time one Gram path on the first batch of a fit (two runs after a warm-up,
// the faster kept); enqueued on the context's stream and synchronized.
static pam_status tune_time(pam_ctx *ctx, FitArgs a, int fused, double *ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    PAM_CHECK_HIP(hipEventCreate(&e0));
    PAM_CHECK_HIP(hipEventCreate(&e1));
    a.gram_fused = fused;
    pam_status st = PAM_OK;
    double best = 1e30;
    for (int rep = 0; rep < 3 && st == PAM_OK; ++rep) {
        if ((st = launch_fill_u32(ctx, ctx->ws.ptr[BUF_FLAGS], 0u, a.n_sub)) != PAM_OK) break;
        (void)hipEventRecord(e0, ctx->stream);
        st = fused ? launch_rowsum(ctx, a) : launch_assemble(ctx, a);
        if (st == PAM_OK) st = fused ? launch_gram_fused(ctx, a) : launch_gram(ctx, a);
        (void)hipEventRecord(e1, ctx->stream);
        if (hipEventSynchronize(e1) != hipSuccess) {
            set_error("tuner: event synchronization failed");
            st = PAM_ERR_HIP;
            break;
        }
        float t = 0.0f;
        (void)hipEventElapsedTime(&t, e0, e1);
        if (rep > 0) best = std::min(best, (double)t);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = best;
    return st;
}

// Path of the plan's Gram: forced by pam_gram_path, else the tuner's choice.
static pam_status tune_gram(pam_ctx *ctx, FitArgs &a, int batch) {
    a.gram_fused = 0;
    if (a.precision == PAM_PREC_F64) return PAM_OK;     // the FP64 design is materialized
    if (ctx->gram_mode == 1) return PAM_OK;
    if (ctx->gram_mode == 2) {
        a.gram_fused = 1;
        return PAM_OK;
    }
    const std::string key = tune_key(a);
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        if (!g_tune_loaded) tune_load();
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            a.gram_fused = it->second.fused;
            return PAM_OK;
        }
    }
    FitArgs t = a;
    t.sub_begin = 0;
    t.sub_count = std::min(batch, a.n_sub);
    t.active = nullptr;
    TuneEntry e{0, 0.0, 0.0};
    pam_status st = tune_time(ctx, t, 0, &e.ms_materialized);
    if (st == PAM_OK) st = tune_time(ctx, t, 1, &e.ms_fused);
    if (st != PAM_OK) return st;
    e.fused = e.ms_fused < e.ms_materialized ? 1 : 0;
    a.gram_fused = e.fused;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    if (g_tune.emplace(key, e).second) tune_store(key, e);
    return PAM_OK;
}

// Launch plan of a3-a6 for subdomains [0, n_sub): the kernel arguments, the
// batch (subdomains per launch, from the workspace budget; batched = 0: one
// per launch) and the solve's team size.
struct FitPlan {
    FitArgs a;
    int batch = 1;
};

static FitPlan fit_plan(const pam_samples *S, const pam_dict *D, const pam_enet_opts *o,
                        double *beta, pam_fit_stats *stats) {
    FitPlan p;
    FitArgs &a = p.a;
    memset(&a, 0, sizeof(a));
    a.n_sub = S->n_sub;
    a.dim = S->dim;
    a.m_cap = D->m_cap;
    a.mpad = mpad_of(D->m_cap);
    a.npad = npad_of(S->n_max);
    a.n_max = S->n_max;
    a.off = S->off;
    a.x = S->x;
    a.y = S->y;
    a.m = D->m;
    a.c = D->c;
    a.sigma = D->sigma;
    a.lambda1 = o->lambda1;
    a.lambda2 = o->lambda2;
    a.lambda1_sub = o->lambda1_sub;
    a.lambda2_sub = o->lambda2_sub;
    a.precision = o->precision;
    a.cd_sweeps = o->cd_sweeps;
    a.max_iter = o->max_iter;
    a.hint = o->support_hint;
    a.beta = beta;
    a.stats = stats;
    a.basis = D->basis;
    a.team = 1;
    a.team_min = o->team_min > 0 ? o->team_min : 128;
    a.team_idle_us = o->team_idle_us;
    const size_t per_sub = (size_t)a.mpad * a.npad * wbytes(a.precision) +
                           (size_t)a.mpad * a.mpad * gbytes(a.precision) +
                           solve_h_elems(a.m_cap) * 8 +
                           solve_scratch_elems(a.m_cap, a.npad, a.precision, 1,
                                               solve_vectors_global(a.m_cap, a.precision)) * 8;
    int batch = o->batched ? (int)std::max<size_t>(1, ws_budget() / std::max<size_t>(per_sub, 1)) : 1;
    p.batch = std::min(batch, a.n_sub);
    if (o->batched) a.team = solve_team_size(p.batch, a.m_cap, a.precision, o->team);
    return p;
}

// Every workspace buffer the plan's launches use, at its final size (so that
// nothing grows while the launches are captured into a graph).
static pam_status fit_ensure(pam_ctx *ctx, const FitPlan &p) {
    const FitArgs &a = p.a;
    const size_t b = (size_t)p.batch;
    pam_status st;
    if ((st = ensure(ctx, BUF_WT, b * a.mpad * a.npad * wbytes(a.precision))) != PAM_OK) return st;
    if ((st = ensure(ctx, BUF_G, b * a.mpad * a.mpad * gbytes(a.precision))) != PAM_OK) return st;
    if ((st = ensure(ctx, BUF_H, b * solve_h_elems(a.m_cap) * 8)) != PAM_OK) return st;
    if ((st = ensure(ctx, BUF_VEC, b * solve_scratch_elems(a.m_cap, a.npad, a.precision, a.team,
                                                          solve_vectors_global(a.m_cap, a.precision)) * 8)) != PAM_OK)
        return st;
    if ((st = ensure(ctx, BUF_FLAGS, (size_t)a.n_sub * 4)) != PAM_OK) return st;
    if (a.team > 1 && (st = ensure(ctx, BUF_TEAM, solve_team_ctl_bytes(p.batch))) != PAM_OK) return st;
    if (a.precision != PAM_PREC_F64 && (st = ensure(ctx, BUF_ROWSUM, b * a.npad * 4)) != PAM_OK) return st;
    return solve_prepare(a.m_cap, a.precision);
}

// fit_ensure, then the Gram path (tuned before any graph capture).
static pam_status fit_prepare(pam_ctx *ctx, FitPlan &p, const double *h) {
    pam_status st = fit_ensure(ctx, p);
    if (st != PAM_OK) return st;
    (void)h;
    return tune_gram(ctx, p.a, p.batch);
}

// Enqueue a3-a6 of the plan: flags cleared, input check, then per batch the
// assembly, the Gram and the solve.
static pam_status fit_enqueue(pam_ctx *ctx, const FitPlan &p, const int32_t *active, int warm_start,
                              const double *h) {
    FitArgs a = p.a;
    a.active = active;
    a.warm_start = warm_start;
    pam_status st;
    if ((st = launch_fill_u32(ctx, ctx->ws.ptr[BUF_FLAGS], 0u, a.n_sub)) != PAM_OK) return st;
    if ((st = launch_check_finite(ctx, a, h)) != PAM_OK) return st;
    for (int b0 = 0; b0 < a.n_sub; b0 += p.batch) {
        a.sub_begin = b0;
        a.sub_count = std::min(p.batch, a.n_sub - b0);
        {
            KernelTimer kt(ctx, PAM_TK_ASSEMBLE);
            if ((st = a.gram_fused ? launch_rowsum(ctx, a) : launch_assemble(ctx, a)) != PAM_OK) return st;
        }
        {
            KernelTimer kt(ctx, PAM_TK_GRAM);
            if ((st = a.gram_fused ? launch_gram_fused(ctx, a) : launch_gram(ctx, a)) != PAM_OK) return st;
        }
        {
            KernelTimer kt(ctx, PAM_TK_SOLVE);
            if ((st = launch_solve(ctx, a)) != PAM_OK) return st;
        }
    }
    return PAM_OK;
}

// Eager a3-a6 (plan, workspace, launches).
static pam_status run_fit(pam_ctx *ctx, const pam_samples *S, const pam_dict *D,
                          const pam_enet_opts *o, double *beta, pam_fit_stats *stats,
                          const int32_t *active, int warm_start, const double *h = nullptr) {
    FitPlan p = fit_plan(S, D, o, beta, stats);
    pam_status st = fit_prepare(ctx, p, h);
    if (st != PAM_OK) return st;
    return fit_enqueue(ctx, p, active, warm_start, h);
}

// ---------------------------------------------------------------- graphs
// FNV-1a over the values that shape a call's launches.
struct KeyHash {
    uint64_t h = 1469598103934665603ull;
    void bytes(const void *p, size_t n) {
        const unsigned char *c = (const unsigned char *)p;
        for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
    }
    template <class T> void v(const T &x) { bytes(&x, sizeof(x)); }
};

static void graph_key_common(KeyHash &k, pam_ctx *ctx, const FitPlan &p, const pam_enet_opts *o) {
    k.v(p.a);   // every kernel argument of the fit (pointers, sizes, parameters, team)
    k.v(p.batch);
    k.v(o->batched);
    for (int b = 0; b < BUF_COUNT; ++b) k.v(ctx->ws.ptr[b]);
    k.v(ctx->sticky);
}

// Runs enqueue() as one HIP graph launch on the context's stream: the
// launches are captured on a private stream into a graph, instantiated and
// kept by key. With kernel timing on, the launches are enqueued directly
// instead (timing events recorded inside a captured graph give no elapsed
// times on this runtime). When a capture cannot be made the work runs
// eagerly with the same launches.
template <class F>
static pam_status graph_run(pam_ctx *ctx, uint64_t key, F &&enqueue) {
    GraphCache &gc = ctx->graphs;
    if (!gc.on || ctx->timing.on) return enqueue();
    hipGraphExec_t exec = nullptr;
    for (auto &e : gc.entries)
        if (e.key == key) {
            exec = e.exec;
            e.used = ++gc.clock;
            break;
        }
    if (!exec) {
        if (!gc.capture) PAM_CHECK_HIP(hipStreamCreateWithFlags(&gc.capture, hipStreamNonBlocking));
        if (hipStreamBeginCapture(gc.capture, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipGetLastError();
            return enqueue();
        }
        const hipStream_t saved = ctx->stream;
        ctx->stream = gc.capture;
        gc.capturing = true;
        const pam_status st = enqueue();
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(gc.capture, &g);
        ctx->stream = saved;
        gc.capturing = false;
        hipError_t ei = hipErrorUnknown;
        if (st == PAM_OK && ec == hipSuccess && g) ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            (void)hipGetLastError();
            exec = nullptr;
            if (st != PAM_OK && st != PAM_ERR_STATE) return st;   // the call itself failed
            return enqueue();                                      // capture not possible: eager
        }
        if (gc.entries.size() >= 16) {
            auto lru = std::min_element(gc.entries.begin(), gc.entries.end(),
                                        [](const GraphCache::Entry &x, const GraphCache::Entry &y) {
                                            return x.used < y.used;
                                        });
            PAM_CHECK_HIP(hipStreamSynchronize(ctx->stream));   // it may still be running
            (void)hipGraphExecDestroy(lru->exec);
            gc.entries.erase(lru);
        }
        gc.entries.push_back({key, exec, ++gc.clock});
    }
    PAM_CHECK_HIP(hipGraphLaunch(exec, ctx->stream));
    return PAM_OK;
}

static pam_status check_fit_args(const pam_samples *S, const pam_dict *D, const pam_enet_opts *o,
                                 const double *beta) {
    PAM_REQUIRE(S && D && o && beta, "NULL argument");
    PAM_REQUIRE(S->dim >= 1 && S->dim <= 3 && S->dim == D->dim, "dimension mismatch");
    PAM_REQUIRE(S->n_sub >= 1 && S->n_sub == D->n_sub, "subdomain count mismatch");
    PAM_REQUIRE(S->off && S->off_host && S->x && S->y, "sample arrays are NULL");
    PAM_REQUIRE(D->m && D->c && D->sigma && D->level, "dictionary arrays are NULL");
    PAM_REQUIRE(D->m_cap >= 1, "m_cap must be >= 1");
    PAM_REQUIRE(D->basis == PAM_BASIS_SHEPARD || D->basis == PAM_BASIS_PLAIN, "unknown basis");
    PAM_REQUIRE(o->lambda1_sub || o->lambda1 >= 0.0, "lambda1 must be >= 0");
    PAM_REQUIRE(o->lambda2_sub || o->lambda2 >= 0.0, "lambda2 must be >= 0");
    PAM_REQUIRE(o->precision >= PAM_PREC_F64 && o->precision <= PAM_PREC_BF16, "unknown precision");
    PAM_REQUIRE(o->cd_sweeps >= 0 && o->max_iter >= 1, "cd_sweeps >= 0 and max_iter >= 1 required");
    PAM_REQUIRE(o->team == 0 || o->team == 1 || o->team == 2 || o->team == 4, "team must be 0, 1, 2 or 4");
    PAM_REQUIRE(o->team_min >= 0, "team_min must be >= 0");
    PAM_REQUIRE(o->team_idle_us >= 0 && o->team_idle_us <= 10000000, "team_idle_us must be in [0, 1e7]");
    int64_t nmax = 0;
    for (int s = 0; s < S->n_sub; ++s) {
        const int64_t n = S->off_host[s + 1] - S->off_host[s];
        PAM_REQUIRE(n >= 0, "sample offsets must be non-decreasing");
        nmax = std::max(nmax, n);
    }
    PAM_REQUIRE(nmax <= S->n_max, "n_max is smaller than the largest subdomain");
    return solve_check_capacity(D->m_cap, o->precision);
}

static pam_status check_ctx(pam_ctx *ctx) {
    if (!ctx || !ctx->alive) {
        set_error("invalid context");
        return PAM_ERR_STATE;
    }
    PAM_CHECK_HIP(hipSetDevice(ctx->device));
    return PAM_OK;
}

}  // namespace pam

using namespace pam;

extern "C" {

const char *pam_last_error(void) { return g_last_error.c_str(); }
const char *pam_version(void) { return "pam-mi355x 0.1 (gfx950)"; }

pam_status pam_create(pam_ctx **out, int device) {
    if (!out) {
        set_error("out is NULL");
        return PAM_ERR_ARG;
    }
    int n = 0;
    PAM_CHECK_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) {
        set_error("no such HIP device");
        return PAM_ERR_ARG;
    }
    PAM_CHECK_HIP(hipSetDevice(device));
    int32_t *sticky = nullptr;
    PAM_CHECK_HIP(hipMalloc(&sticky, 4 * sizeof(int32_t)));
    if (hipMemset(sticky, 0, 4 * sizeof(int32_t)) != hipSuccess) {
        (void)hipFree(sticky);
        set_error("pam_create: hipMemset failed");
        return PAM_ERR_HIP;
    }
    pam_status sst = eval_scratch_init(device);   // once per device: pam_eval_noalloc's array
    if (sst != PAM_OK) {
        (void)hipFree(sticky);
        return sst;
    }
    pam_ctx *c = new pam_ctx();
    c->device = device;
    c->sticky = sticky;
    *out = c;
    return PAM_OK;
}

pam_status pam_destroy(pam_ctx *ctx) {
    if (!ctx) return PAM_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &e : ctx->graphs.entries) (void)hipGraphExecDestroy(e.exec);
    ctx->graphs.entries.clear();
    if (ctx->graphs.capture) (void)hipStreamDestroy(ctx->graphs.capture);
    for (int b = 0; b < BUF_COUNT; ++b)
        if (ctx->ws.ptr[b]) (void)hipFree(ctx->ws.ptr[b]);
    for (auto &p : ctx->timing.pending) {
        (void)hipEventDestroy(p.second.first);
        (void)hipEventDestroy(p.second.second);
    }
    for (hipEvent_t e : ctx->timing.pool) (void)hipEventDestroy(e);
    if (ctx->staging.host) (void)hipHostFree(ctx->staging.host);
    if (ctx->staging.done) (void)hipEventDestroy(ctx->staging.done);
    if (ctx->sticky) (void)hipFree(ctx->sticky);
    ctx->alive = false;
    delete ctx;
    return PAM_OK;
}

pam_status pam_set_stream(pam_ctx *ctx, void *stream) {
    pam_status st = check_ctx(ctx);
    if (st != PAM_OK) return st;
    ctx->stream = (hipStream_t)stream;
    return PAM_OK;
}

pam_status pam_sync(pam_ctx *ctx) {
    pam_status st = check_ctx(ctx);
    if (st != PAM_OK) return st;
    PAM_CHECK_HIP(hipStreamSynchronize(ctx->stream));
    int32_t bad = 0;
    PAM_CHECK_HIP(hipMemcpy(&bad, ctx->sticky, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (bad) {
        PAM_CHECK_HIP(hipMemsetAsync(ctx->sticky, 0, sizeof(int32_t), ctx->stream));
        PAM_CHECK_HIP(hipStreamSynchronize(ctx->stream));
        set_error("non-finite input (or a width <= 0) in " + std::to_string(bad) +
                  " subdomain fit(s) since the previous pam_sync; see the per-subdomain status");
        return PAM_ERR_NONFINITE;
    }
    return PAM_OK;
}

pam_status pam_gram_path(pam_ctx *ctx, int32_t mode) {
    pam_status st = check_ctx(ctx);
    if (st != PAM_OK) return st;
    PAM_REQUIRE(mode >= 0 && mode <= 2, "mode must be 0 (tuned), 1 (materialized) or 2 (fused)");
    ctx->gram_mode = mode;
    return PAM_OK;
}

pam_status pam_graph_enable(pam_ctx *ctx, int32_t on) {
    pam_status st = check_ctx(ctx);
    if (st != PAM_OK) return st;
    ctx->graphs.on = on != 0;
    return PAM_OK;
}

pam_status pam_timing_enable(pam_ctx *ctx, int32_t on) {
    pam_status st = check_ctx(ctx);
    if (st != PAM_OK) return st;
    ctx->timing.on = on != 0;
    return PAM_OK;
}

pam_status pam_timing_read(pam_ctx *ctx, double *ms, int64_t *launches, int32_t reset) {
    pam_status st = check_ctx(ctx);
    if (st != PAM_OK) return st;
    PAM_REQUIRE(ms && launches, "NULL output");
    Timing &t = ctx->timing;
    PAM_CHECK_HIP(hipStreamSynchronize(ctx->stream));
    for (auto &p : t.pending) {
        float e = 0.0f;
        PAM_CHECK_HIP(hipEventElapsedTime(&e, p.second.first, p.second.second));
        t.ms[p.first] += e;
        t.count[p.first] += 1;
        t.pool.push_back(p.second.first);
        t.pool.push_back(p.second.second);
    }
    t.pending.clear();
    for (int k = 0; k < PAM_TK_COUNT; ++k) {
        ms[k] = t.ms[k];
        launches[k] = t.count[k];
        if (reset) {
            t.ms[k] = 0.0;
            t.count[k] = 0;
        }
    }
    return PAM_OK;
}

pam_status pam_partition_count(const pam_grid *grid, int64_t *off_host, int32_t *n_max) {
    int n_sub = 0;
    pam_status st = check_grid(grid, &n_sub);
    if (st != PAM_OK) return st;
    PAM_REQUIRE(off_host && n_max, "NULL output");
    std::vector<char> tab(gather_table_bytes(n_sub));
    build_gather_table(grid, tab.data());
    const int32_t *t = (const int32_t *)tab.data();  // first[3], last[3] per subdomain
    off_host[0] = 0;
    int64_t mx = 0;
    for (int s = 0; s < n_sub; ++s) {
        int64_t cnt = 1;
        for (int a = 0; a < grid->dim; ++a) cnt *= (int64_t)(t[s * 6 + 3 + a] - t[s * 6 + a]);
        off_host[s + 1] = off_host[s] + cnt;
        mx = std::max(mx, cnt);
    }
    *n_max = (int32_t)mx;
    return PAM_OK;
}

pam_status pam_partition_gather(pam_ctx *ctx, const pam_grid *grid, const double *cell_y,
                                const int64_t *off, double *x, double *y, double *h, int32_t *cell) {
    pam_status st = check_ctx(ctx);
    if (st != PAM_OK) return st;
    int n_sub = 0;
    if ((st = check_grid(grid, &n_sub)) != PAM_OK) return st;
    PAM_REQUIRE(cell_y && off && x && y && h && cell, "NULL argument");
    std::vector<int64_t> offh(n_sub + 1);
    int32_t n_max = 0;
    if ((st = pam_partition_count(grid, offh.data(), &n_max)) != PAM_OK) return st;
    std::vector<char> tab(gather_table_bytes(n_sub));
    build_gather_table(grid, tab.data());
    if ((st = upload(ctx, BUF_TABLE, tab.data(), tab.size())) != PAM_OK) return st;
    KernelTimer kt(ctx, PAM_TK_GATHER);
    return launch_gather(ctx, grid, ctx->ws.ptr[BUF_TABLE], n_sub, n_max, cell_y, off, x, y, h, cell);
}

pam_status pam_init_lattice(pam_ctx *ctx, const pam_grid *grid, const int32_t *g,
                            double sigma_factor, pam_dict *dict) {
    pam_status st = check_ctx(ctx);
    if (st != PAM_OK) return st;
    int n_sub = 0;
    if ((st = check_grid(grid, &n_sub)) != PAM_OK) return st;
    PAM_REQUIRE(g && dict && dict->m && dict->c && dict->sigma && dict->level, "NULL argument");
    PAM_REQUIRE(dict->n_sub == n_sub && dict->dim == grid->dim, "dictionary does not match grid");
    PAM_REQUIRE(sigma_factor > 0.0, "sigma_factor must be > 0");
    int64_t M = 1;
    for (int a = 0; a < grid->dim; ++a) {
        PAM_REQUIRE(g[a] >= 1, "lattice counts must be >= 1");
        M *= g[a];
    }
    if (M > dict->m_cap) {
        set_error("m_cap too small for the lattice: need " + std::to_string(M));
        return PAM_ERR_CAPACITY;
    }
    std::vector<char> tab(lattice_table_bytes(n_sub));
    build_lattice_table(grid, g, sigma_factor, tab.data());
    if ((st = upload(ctx, BUF_TABLE, tab.data(), tab.size())) != PAM_OK) return st;
    KernelTimer kt(ctx, PAM_TK_LATTICE);
    return launch_lattice(ctx, grid->dim, g, n_sub, dict->m_cap, ctx->ws.ptr[BUF_TABLE], dict);
}

pam_status pam_fit_subdomains(pam_ctx *ctx, const pam_samples *samples, const pam_dict *dict,
                              const pam_enet_opts *opts, double *beta, pam_fit_stats *stats) {
    pam_status st = check_ctx(ctx);
    if (st != PAM_OK) return st;
    if ((st = check_fit_args(samples, dict, opts, beta)) != PAM_OK) return st;
    FitPlan plan = fit_plan(samples, dict, opts, beta, stats);
    if ((st = fit_prepare(ctx, plan, nullptr)) != PAM_OK) return st;
    KeyHash k;
    k.v(1);   // a single fit
    graph_key_common(k, ctx, plan, opts);
    k.v(opts->warm_start);
    return graph_run(ctx, k.h, [&]() { return fit_enqueue(ctx, plan, nullptr, opts->warm_start, nullptr); });
}

pam_status pam_refit_nonconverged(pam_ctx *ctx, const pam_samples *samples, const pam_dict *dict,
                                  const pam_enet_opts *opts, double *beta, pam_fit_stats *stats) {
    pam_status st = check_ctx(ctx);
    if (st != PAM_OK) return st;
    PAM_REQUIRE(opts, "NULL argument");
    PAM_REQUIRE(stats, "stats is NULL: the refit reads the statuses of the previous fit");
    pam_enet_opts o = *opts;
    o.precision = PAM_PREC_F64;
    o.warm_start = 0;
    o.support_hint = nullptr;
    if ((st = check_fit_args(samples, dict, &o, beta)) != PAM_OK) return st;
    const int n = samples->n_sub;
    if ((st = ensure(ctx, BUF_TABLE, (size_t)n * 4)) != PAM_OK) return st;
    int32_t *mask = wsp<int32_t>(ctx, BUF_TABLE);
    if ((st = launch_noconv_mask(ctx, stats, n, mask)) != PAM_OK) return st;
    return run_fit(ctx, samples, dict, &o, beta, stats, mask, 0);
}

pam_status pam_refine(pam_ctx *ctx, const pam_samples *samples, pam_dict *dict, double *beta,
                      const pam_enet_opts *opts, const pam_refine_opts *r, pam_fit_stats *stats) {
    pam_status st = check_ctx(ctx);
    if (st != PAM_OK) return st;
    if ((st = check_fit_args(samples, dict, opts, beta)) != PAM_OK) return st;
    PAM_REQUIRE(r && r->elem_level && samples->h, "refinement arguments are NULL");
    PAM_REQUIRE(r->max_rounds >= 0 && r->m_max >= 0, "max_rounds and m_max must be >= 0");
    PAM_REQUIRE(r->eta > 0.0 && r->eta < 1.0, "eta must be in (0, 1)");
    PAM_REQUIRE(r->k_top >= 0 || r->k_top_sub, "k_top must be >= 0");
    PAM_REQUIRE(r->space == 0 || r->space == 1, "space must be 0 or 1");
    if ((st = mark_check_capacity(samples->n_max)) != PAM_OK) return st;
    const int n = samples->n_sub;
    // per-subdomain int tables: active, m0, k_top (uploaded before the
    // rounds; the rounds themselves are one graph launch)
    std::vector<int32_t> tab((size_t)3 * n);
    for (int s = 0; s < n; ++s) {
        tab[s] = 1;
        tab[2 * n + s] = r->k_top_sub ? r->k_top_sub[s] : r->k_top;
    }
    if ((st = upload(ctx, BUF_TABLE, tab.data(), tab.size() * 4)) != PAM_OK) return st;
    int32_t *active = wsp<int32_t>(ctx, BUF_TABLE);
    int32_t *m0 = active + n;
    int32_t *ktop = active + 2 * n;
    const int64_t n_tot = samples->off_host[n];
    if ((st = ensure(ctx, BUF_R, (size_t)std::max<int64_t>(n_tot, 1) * 8)) != PAM_OK) return st;
    if ((st = ensure(ctx, BUF_MARK, mark_ws_bytes(n, samples->n_max))) != PAM_OK) return st;
    FitPlan plan = fit_plan(samples, dict, opts, beta, stats);
    if ((st = fit_prepare(ctx, plan, samples->h)) != PAM_OK) return st;
    RefineArgs ra;
    memset(&ra, 0, sizeof(ra));
    ra.n_sub = n;
    ra.dim = samples->dim;
    ra.m_cap = dict->m_cap;
    ra.n_max = samples->n_max;
    ra.off = samples->off;
    ra.x = samples->x;
    ra.y = samples->y;
    ra.h = samples->h;
    ra.m = dict->m;
    ra.c = dict->c;
    ra.sigma = dict->sigma;
    ra.level = dict->level;
    ra.beta = beta;
    ra.k_top = ktop;
    ra.m_max = r->m_max;
    ra.space = r->space;
    ra.max_rounds = r->max_rounds;
    ra.eta = r->eta;
    ra.eps_tol = r->eps_tol;
    ra.elem_level = r->elem_level;
    ra.active = active;
    ra.m0 = m0;
    ra.rounds = r->rounds;
    ra.round_stats = r->round_stats;
    ra.stats = stats;
    ra.basis = dict->basis;
    ra.flags = wsp<int32_t>(ctx, BUF_FLAGS);
    // every round is enqueued up front: subdomains that stop clear their
    // active flag on the device and every later kernel skips them
    auto rounds = [&]() -> pam_status {
        pam_status s2;
        if ((s2 = launch_copy_i32(ctx, m0, dict->m, n)) != PAM_OK) return s2;
        for (int round = 0; round <= r->max_rounds; ++round) {
            const int warm = round == 0 ? opts->warm_start : (r->cold_rounds ? 0 : 1);
            if ((s2 = fit_enqueue(ctx, plan, active, warm, samples->h)) != PAM_OK) return s2;
            RefineArgs rr = ra;
            rr.round = round;
            {
                KernelTimer kt(ctx, PAM_TK_INDICATOR);
                if ((s2 = launch_indicator(ctx, rr)) != PAM_OK) return s2;
            }
            {
                KernelTimer kt(ctx, PAM_TK_MARK);
                if ((s2 = launch_mark_enrich(ctx, rr)) != PAM_OK) return s2;
            }
        }
        return PAM_OK;
    };
    KeyHash k;
    k.v(2);   // a refinement
    graph_key_common(k, ctx, plan, opts);
    k.v(ra);
    k.v(opts->warm_start);
    k.v(r->cold_rounds);
    return graph_run(ctx, k.h, rounds);
}

pam_status pam_select_lambda(pam_ctx *ctx, const pam_samples *samples, const pam_dict *dict,
                             const pam_enet_opts *opts, const pam_select_opts *sel, double *alpha,
                             double *score, int32_t *best, double *lambda1_sub,
                             double *lambda2_sub, int32_t *n_failed) {
    pam_status st = check_ctx(ctx);
    if (st != PAM_OK) return st;
    PAM_REQUIRE(opts && sel && alpha && score && best && lambda1_sub && lambda2_sub,
                "NULL argument");
    PAM_REQUIRE(sel->n_alpha >= 1 && sel->n_alpha <= 4096, "n_alpha must be in [1, 4096]");
    PAM_REQUIRE(sel->k_folds >= 2 && sel->k_folds <= 64, "k_folds must be in [2, 64]");
    PAM_REQUIRE(sel->alpha_min_ratio > 0.0 && sel->alpha_min_ratio <= 1.0,
                "alpha_min_ratio must be in (0, 1]");
    PAM_REQUIRE(sel->l1_ratio > 0.0 && sel->l1_ratio <= 1.0, "l1_ratio must be in (0, 1]");
    pam_enet_opts o = *opts;   // the path sets the parameters; a hint does not apply
    o.lambda1 = o.lambda2 = 0.0;
    o.lambda1_sub = o.lambda2_sub = nullptr;
    o.support_hint = nullptr;
    if ((st = check_fit_args(samples, dict, &o, alpha)) != PAM_OK) return st;
    const int n = samples->n_sub, K = sel->k_folds, nv = n * K, dim = samples->dim;
    const int m_cap = dict->m_cap;
    // training sets: fold f of subdomain s holds its samples j with j % K == f
    std::vector<int64_t> off_v((size_t)nv + 1, 0);
    int n_max_v = 0;
    for (int s = 0; s < n; ++s) {
        const int64_t N = samples->off_host[s + 1] - samples->off_host[s];
        for (int f = 0; f < K; ++f) {
            const int64_t held = N > f ? (N - 1 - f) / K + 1 : 0;
            const int64_t cnt = N - held;
            off_v[(size_t)s * K + f + 1] = off_v[(size_t)s * K + f] + cnt;
            n_max_v = std::max<int>(n_max_v, (int)cnt);
        }
    }
    const int64_t n_tot = samples->off_host[n];
    const int64_t n_tot_v = off_v[nv];
    size_t w = 0;
    auto take = [&](size_t bytes) { size_t r = w; w += (bytes + 255) / 256 * 256; return r; };
    const size_t o_off = take(sizeof(int64_t) * (nv + 1));
    const size_t o_x = take(sizeof(double) * std::max<int64_t>(n_tot_v, 1) * dim);
    const size_t o_y = take(sizeof(double) * std::max<int64_t>(n_tot_v, 1));
    const size_t o_m = take(sizeof(int32_t) * nv);
    const size_t o_c = take(sizeof(double) * (size_t)nv * m_cap * dim);
    const size_t o_s = take(sizeof(double) * (size_t)nv * m_cap);
    const size_t o_l = take(sizeof(int32_t) * (size_t)nv * m_cap);
    const size_t o_b = take(sizeof(double) * (size_t)nv * m_cap);
    const size_t o_l1 = take(sizeof(double) * nv);
    const size_t o_l2 = take(sizeof(double) * nv);
    const size_t o_st = take(sizeof(pam_fit_stats) * nv);
    const size_t o_inv = take(sizeof(double) * std::max<int64_t>(n_tot, 1));
    if ((st = ensure(ctx, BUF_EVAL, w)) != PAM_OK) return st;
    char *base = wsp<char>(ctx, BUF_EVAL);
    if ((st = upload_to(ctx, base + o_off, off_v.data(), sizeof(int64_t) * (nv + 1))) != PAM_OK)
        return st;
    pam_samples Sv;
    memset(&Sv, 0, sizeof(Sv));
    Sv.dim = dim;
    Sv.n_sub = nv;
    Sv.n_max = n_max_v;
    Sv.off = (const int64_t *)(base + o_off);
    Sv.off_host = off_v.data();
    Sv.x = (const double *)(base + o_x);
    Sv.y = (const double *)(base + o_y);
    pam_dict Dv;
    memset(&Dv, 0, sizeof(Dv));
    Dv.n_sub = nv;
    Dv.dim = dim;
    Dv.m_cap = m_cap;
    Dv.m = (int32_t *)(base + o_m);
    Dv.c = (double *)(base + o_c);
    Dv.sigma = (double *)(base + o_s);
    Dv.level = (int32_t *)(base + o_l);
    Dv.basis = dict->basis;
    double *beta_v = (double *)(base + o_b);
    double *l1v = (double *)(base + o_l1);
    double *l2v = (double *)(base + o_l2);
    pam_fit_stats *stats_v = (pam_fit_stats *)(base + o_st);
    const double rho = sel->l1_ratio;
    if ((st = launch_cv_setup(ctx, samples, dict, K, Sv.off, (double *)Sv.x, (double *)Sv.y, Dv.m,
                              Dv.c, Dv.sigma, Dv.level, beta_v, (double *)(base + o_inv),
                              sel->n_alpha, sel->alpha_min_ratio, rho, alpha, n_failed)) != PAM_OK)
        return st;
    o.lambda1_sub = l1v;
    o.lambda2_sub = l2v;
    for (int k = 0; k < sel->n_alpha; ++k) {
        if ((st = launch_cv_lambda(ctx, n, K, sel->n_alpha, k, rho, alpha, l1v, l2v)) != PAM_OK)
            return st;
        // path order: each fit starts from the previous alpha's solution
        if ((st = run_fit(ctx, &Sv, &Dv, &o, beta_v, stats_v, nullptr, k > 0 ? 1 : 0)) != PAM_OK)
            return st;
        if ((st = launch_cv_score(ctx, samples, dict, K, sel->n_alpha, k, beta_v, stats_v, score,
                                  n_failed)) != PAM_OK)
            return st;
    }
    // the host offsets above are read by run_fit during the calls only
    return launch_cv_choose(ctx, n, sel->n_alpha, rho, alpha, score, best, lambda1_sub,
                            lambda2_sub);
}

static pam_status check_darcy(const pam_darcy_opts *o) {
    PAM_REQUIRE(o, "NULL options");
    PAM_REQUIRE(o->n[0] >= 1 && o->n[1] >= 1, "n must be >= 1");
    PAM_REQUIRE((int64_t)(o->n[0] + 1) * (o->n[1] + 1) <= ((int64_t)1 << 30), "mesh too large");
    PAM_REQUIRE(o->hi[0] > o->lo[0] && o->hi[1] > o->lo[1], "the box needs lo < hi");
    PAM_REQUIRE(o->tol > 0.0 && o->max_iter >= 1 && o->check_every >= 1,
                "tol > 0, max_iter >= 1 and check_every >= 1 required");
    return PAM_OK;
}

pam_status pam_darcy_solve(pam_ctx *ctx, const pam_darcy_opts *opts, const double *k_tri,
                           double *p, int32_t warm, int32_t *iters, double *rel_res) {
    pam_status st = check_ctx(ctx);
    if (st != PAM_OK) return st;
    if ((st = check_darcy(opts)) != PAM_OK) return st;
    PAM_REQUIRE(k_tri && p && iters && rel_res, "NULL argument");
    return launch_darcy_solve(ctx, opts, k_tri, p, warm ? 1 : 0, iters, rel_res);
}

pam_status pam_darcy_error(pam_ctx *ctx, const pam_darcy_opts *opts, const double *p_ref,
                           const double *p, double *e_rel) {
    pam_status st = check_ctx(ctx);
    if (st != PAM_OK) return st;
    if ((st = check_darcy(opts)) != PAM_OK) return st;
    PAM_REQUIRE(p_ref && p && e_rel, "NULL argument");
    return launch_darcy_error(ctx, opts, p_ref, p, e_rel);
}

// Field table checks shared by the evaluation entry points; with Q < 0 the
// query ranges are not checked (interface jump).
static pam_status check_fields(int32_t n_fields, const pam_field *fields, const pam_dict *dict,
                               int64_t Q) {
    PAM_REQUIRE(n_fields >= 1 && fields && dict, "NULL argument");
    int64_t prev = 0;
    for (int f = 0; f < n_fields; ++f) {
        const pam_field &F = fields[f];
        PAM_REQUIRE(F.dim == dict->dim && F.axis_x, "field dimension mismatch");
        if (Q >= 0) {
            PAM_REQUIRE(F.q_begin == prev && F.q_end >= F.q_begin && F.q_end <= Q,
                        "field query ranges must tile [0, Q) in order");
            prev = F.q_end;
        }
        int nsub = 1, pos = 0;
        for (int d = 0; d < F.dim; ++d) {
            PAM_REQUIRE(F.n_sub_axis[d] >= 1, "n_sub_axis must be >= 1");
            for (int i = 0; i < F.n_sub_axis[d]; ++i)
                PAM_REQUIRE(F.axis_x[pos + i + 1] > F.axis_x[pos + i], "axis breakpoints must increase");
            pos += F.n_sub_axis[d] + 1;
            nsub *= F.n_sub_axis[d];
        }
        PAM_REQUIRE(F.sub_base >= 0 && F.sub_base + nsub <= dict->n_sub,
                    "field subdomains exceed the dictionary");
    }
    if (Q >= 0) PAM_REQUIRE(prev == Q, "field query ranges must cover [0, Q)");
    return PAM_OK;
}

pam_status pam_eval(pam_ctx *ctx, int32_t n_fields, const pam_field *fields, const pam_dict *dict,
                    const double *beta, int32_t dtype, const void *xq, int64_t Q, void *out,
                    int32_t space, int64_t *n_outside) {
    pam_status st = check_ctx(ctx);
    if (st != PAM_OK) return st;
    PAM_REQUIRE(beta, "NULL argument");
    PAM_REQUIRE(Q >= 0 && (Q == 0 || (xq && out)), "query arrays are NULL");
    PAM_REQUIRE(dtype == 0 || dtype == 1, "dtype must be 0 (f32) or 1 (f64)");
    PAM_REQUIRE(space == 0 || space == 1, "space must be 0 or 1");
    if ((st = check_fields(n_fields, fields, dict, Q)) != PAM_OK) return st;
    return launch_eval(ctx, n_fields, fields, dict, beta, dtype, xq, Q, out, space, n_outside);
}

pam_status pam_eval_noalloc(pam_ctx *ctx, int32_t n_fields, const pam_field *fields,
                            const pam_dict *dict, const double *beta, int32_t dtype, const void *xq,
                            int64_t Q, void *out, int32_t space, int64_t *n_outside) {
    pam_status st = check_ctx(ctx);
    if (st != PAM_OK) return st;
    PAM_REQUIRE(beta, "NULL argument");
    PAM_REQUIRE(Q >= 0 && (Q == 0 || (xq && out)), "query arrays are NULL");
    PAM_REQUIRE(dtype == 0 || dtype == 1, "dtype must be 0 (f32) or 1 (f64)");
    PAM_REQUIRE(space == 0 || space == 1, "space must be 0 or 1");
    if ((st = check_fields(n_fields, fields, dict, Q)) != PAM_OK) return st;
    return launch_eval_noalloc(ctx, n_fields, fields, dict, beta, dtype, xq, Q, out, space, n_outside);
}

pam_status pam_eval_blend(pam_ctx *ctx, int32_t n_fields, const pam_field *fields,
                          const pam_dict *dict, const double *beta, double blend, int32_t dtype,
                          const void *xq, int64_t Q, void *out, int32_t space,
                          int64_t *n_outside) {
    pam_status st = check_ctx(ctx);
    if (st != PAM_OK) return st;
    PAM_REQUIRE(beta, "NULL argument");
    PAM_REQUIRE(blend >= 0.0 && blend <= 0.5, "blend must be in [0, 1/2]");
    PAM_REQUIRE(Q >= 0 && (Q == 0 || (xq && out)), "query arrays are NULL");
    PAM_REQUIRE(dtype == 0 || dtype == 1, "dtype must be 0 (f32) or 1 (f64)");
    PAM_REQUIRE(space == 0 || space == 1, "space must be 0 or 1");
    if ((st = check_fields(n_fields, fields, dict, Q)) != PAM_OK) return st;
    PAM_REQUIRE(Q <= ((int64_t)1 << 59), "too many queries");
    return launch_eval_blend(ctx, n_fields, fields, dict, beta, blend, dtype, xq, Q, out, space,
                             n_outside);
}

pam_status pam_darcy_coefficient(pam_ctx *ctx, const pam_darcy_opts *opts, const pam_field *field,
                                 const pam_dict *dict, const double *beta, double blend,
                                 double *k_tri) {
    pam_status st = check_ctx(ctx);
    if (st != PAM_OK) return st;
    if ((st = check_darcy(opts)) != PAM_OK) return st;
    PAM_REQUIRE(field && dict && beta && k_tri, "NULL argument");
    PAM_REQUIRE(field->dim == 2, "the Darcy mesh is two-dimensional");
    PAM_REQUIRE(blend < 0.0 || blend <= 0.5, "blend must be < 0 (owner) or in [0, 1/2]");
    pam_field f = *field;
    const int64_t Q = 2 * (int64_t)opts->n[0] * opts->n[1];
    f.q_begin = 0;
    f.q_end = Q;
    if ((st = check_fields(1, &f, dict, Q)) != PAM_OK) return st;
    return launch_darcy_coefficient(ctx, opts, &f, dict, beta, blend, k_tri);
}

pam_status pam_darcy_coefficient_cells(pam_ctx *ctx, const pam_darcy_opts *opts,
                                       const double *cell_y, double *k_tri) {
    pam_status st = check_ctx(ctx);
    if (st != PAM_OK) return st;
    if ((st = check_darcy(opts)) != PAM_OK) return st;
    PAM_REQUIRE(cell_y && k_tri, "NULL argument");
    return launch_darcy_cells(ctx, opts, cell_y, k_tri);
}

int64_t pam_interface_count(int32_t n_fields, const pam_field *fields) {
    if (n_fields < 1 || !fields) return -1;
    for (int f = 0; f < n_fields; ++f) {
        if (fields[f].dim < 1 || fields[f].dim > 3) return -1;
        for (int d = 0; d < fields[f].dim; ++d)
            if (fields[f].n_sub_axis[d] < 1) return -1;
    }
    return interface_count(n_fields, fields);
}

pam_status pam_interface_jump(pam_ctx *ctx, int32_t n_fields, const pam_field *fields,
                              const pam_dict *dict, const double *beta, int32_t n_per_axis,
                              double *out) {
    pam_status st = check_ctx(ctx);
    if (st != PAM_OK) return st;
    PAM_REQUIRE(beta, "NULL argument");
    PAM_REQUIRE(n_per_axis >= 1 && n_per_axis <= 4096, "n_per_axis must be in [1, 4096]");
    if ((st = check_fields(n_fields, fields, dict, -1)) != PAM_OK) return st;
    const int64_t nf = interface_count(n_fields, fields);
    PAM_REQUIRE(nf == 0 || out, "out is NULL");
    int64_t pts = 1;
    for (int d = 0; d + 1 < dict->dim; ++d) pts *= n_per_axis;
    PAM_REQUIRE(pts <= ((int64_t)1 << 24), "too many samples per face");
    PAM_REQUIRE(nf < ((int64_t)1 << 31), "too many interfaces");
    return launch_interface_jump(ctx, n_fields, fields, dict, beta, n_per_axis, out);
}

}  // extern "C"
