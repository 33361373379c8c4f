/*
 * pam.h -- C ABI of the MI355X (gfx950) implementation of the PAM
 * reconstruction hot path: Parallel and Adaptive Mesh-free approximation of
 * cellwise-constant coefficient data by Shepard-normalized Gaussian RBF
 * expansions fitted per subdomain with an elastic net, residual-driven
 * enrichment, and evaluation of the closed-form field at arbitrary points.
 *
 * Conventions for every entry point:
 *  - Pointers are DEVICE pointers unless the comment says [host].
 *  - The caller allocates and frees every buffer it passes; the library never
 *    frees caller memory. The context owns its workspace (grown on demand
 *    with hipMalloc) and its launch caches.
 *  - Work is enqueued asynchronously on the context's stream (pam_set_stream).
 *    Argument errors are detected on the host and returned before anything is
 *    enqueued; data-dependent conditions (non-convergence, denominator
 *    underflow) are reported per subdomain in the stats arrays.
 *  - Return values are pam_status codes; pam_last_error() gives a message for
 *    the last failing call on the calling thread. No C++ exception crosses the
 *    ABI. A context is not thread-safe.
 *  - Floating-point inputs are FP64. Subdomains are numbered row-major over
 *    the subdomain grid with axis 0 fastest; samples of a subdomain are
 *    contiguous (CSR offsets) in the same row-major cell order.
 *  - Dictionaries are capacity-padded: subdomain s owns the slots
 *    [s*m_cap, (s+1)*m_cap) of sigma/level/beta and [s*m_cap*dim, ...) of c.
 */
#ifndef PAM_H
#define PAM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PAM_OK = 0,
    PAM_ERR_ARG = -1,       /* invalid argument (shape, range, NULL)          */
    PAM_ERR_CAPACITY = -2,  /* a capacity (m_cap, workspace cap) is too small */
    PAM_ERR_NONFINITE = -3, /* pam_sync only: since the previous pam_sync a fit
                               met a sample point, data value, center or width
                               that is NaN or infinite (or a width <= 0); the
                               subdomains concerned carry PAM_ST_NONFINITE   */
    PAM_ERR_HIP = -5,       /* a HIP runtime call failed                      */
    PAM_ERR_NOMEM = -6,     /* workspace allocation failed                    */
    PAM_ERR_STATE = -7      /* context not usable (destroyed, wrong device)   */
} pam_status;

/* Per-subdomain status written to pam_fit_stats.status. */
enum {
    PAM_ST_OK = 0,
    PAM_ST_NOCONV = 1,     /* active-set iteration cap reached / singular block */
    PAM_ST_UNDERFLOW = 2,  /* a Shepard denominator was not a positive normal   */
    PAM_ST_EMPTY = 3,      /* subdomain without samples or centers              */
    PAM_ST_NONFINITE = 4   /* a sample point, data value, element extent (refine),
                              center or width of the subdomain is NaN or
                              infinite, or a width is <= 0: the subdomain is not
                              fitted (beta = 0) and, in pam_refine, not refined.
                              The paper's data are positive coefficients whose
                              logarithm is fitted (remark after Sec. 3.3), so a
                              non-finite value has no meaning for the method  */
};

/* Precision of the normalized design and of its Gram products. The
 * active-support solve, its residual refinement and the KKT certificate are
 * FP64 in every mode. The FP32 and BF16 modes start the FP64 refinement from
 * the active set the low-precision Gram settles on; that start is close on
 * the Shepard basis, but on far worse conditioned active blocks (the
 * unnormalized basis, PAM_BASIS_PLAIN, on refined dictionaries) the FP64
 * refinement can reach its iteration cap first. Such a subdomain reports
 * PAM_ST_NOCONV with the coefficients it reached; pam_refit_nonconverged fits
 * exactly those subdomains again with the FP64 Gram. */
typedef enum {
    PAM_PREC_F64 = 0,   /* FP64 design, FP64 MFMA Gram                         */
    PAM_PREC_F32 = 1,   /* FP32 design, FP32 MFMA Gram, FP64 refinement        */
    PAM_PREC_BF16 = 2   /* BF16 design, BF16 MFMA Gram with FP32 accumulation  */
} pam_precision;

typedef struct pam_ctx pam_ctx;

/* Create a context bound to HIP device `device`. */
pam_status pam_create(pam_ctx **out, int device);
/* Release the context and its workspace (synchronizes its stream first). */
pam_status pam_destroy(pam_ctx *ctx);
/* Stream used for all later calls (a hipStream_t; NULL = the null stream). */
pam_status pam_set_stream(pam_ctx *ctx, void *stream);
/* Block until all work enqueued by the context has finished. Returns
 * PAM_ERR_NONFINITE if any fit enqueued since the previous pam_sync met
 * non-finite input (a sticky device flag, cleared by this call; the
 * per-subdomain status says which subdomains), else PAM_OK or PAM_ERR_HIP. */
pam_status pam_sync(pam_ctx *ctx);
/* Batched launches as HIP graphs (default on): pam_fit_subdomains and
 * pam_refine capture all of their launches (every round of a refinement,
 * with the per-subdomain active flags the kernels read on the device: a
 * subdomain that stops is skipped by every later launch) into one graph on a
 * private stream, instantiate it once per call shape (pointers, sizes,
 * options and workspace addresses) and replay it with one hipGraphLaunch on
 * the context's stream. While kernel timing is on (pam_timing_enable), and
 * with on = 0, the same launches are enqueued directly. Results are
 * identical either way. */
pam_status pam_graph_enable(pam_ctx *ctx, int32_t on);
/* Path of the FP32 / BF16 Gram products (a5 with a3-a4): 1 = the assembly
 * writes the normalized design W to HBM and the MFMA Gram tiles read it;
 * 2 = fused: the Shepard denominators are computed first, then every Gram
 * tile computes the design entries it needs in LDS and contracts them on
 * MFMA, so W never reaches HBM; 0 (default) = tuned: both are timed on the
 * first batched fit of each (precision, padded M, padded N) bucket and the
 * faster is kept for the process (and appended to the JSON-lines file
 * PAM_TUNE_CACHE names, read back at the first lookup). The two paths give
 * bit-identical Gram products. FP64 always uses the stored design. */
pam_status pam_gram_path(pam_ctx *ctx, int32_t mode);
/* [host] Message of the last failing call on this thread ("" if none). */
const char *pam_last_error(void);
/* [host] Library version string. */
const char *pam_version(void);

/* ------------------------------------------------------------------------
 * a1. Structured grid and box partition (Sec. 2 Step 1: half-open
 * non-overlapping subdomains, every element in exactly one; Step 2: one
 * sample per element at its centroid). With overlap > 0 the fit set of a
 * subdomain is widened by overlap * width on interior faces; ownership for
 * evaluation stays half-open.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t dim;            /* 1, 2 or 3                                      */
    int32_t n_cells[3];     /* cells per axis (unused axes: 1)                */
    double lo[3], hi[3];    /* domain box                                     */
    int32_t n_sub[3];       /* subdomains per axis (unused axes: 1)           */
    const int32_t *breaks;  /* [host] per-axis cell-index breakpoints,
                               concatenated: n_sub[a]+1 strictly increasing
                               values from 0 to n_cells[a] for each axis      */
    double overlap;         /* >= 0, fraction of the subdomain width          */
} pam_grid;

/* [host] Sample counts: off_host[0..n_sub_total] (CSR offsets, int64) of the
 * partition; *n_max = largest subdomain sample count. No device work. */
pam_status pam_partition_count(const pam_grid *grid, int64_t *off_host, int32_t *n_max);

/* a1 on the device: gather centroids x [N_tot*dim], values y [N_tot],
 * element extents h [N_tot*dim] and integer cell indices cell [N_tot*dim]
 * from the cell values cell_y [n_cells product, axis 0 fastest].
 * off: device copy of the offsets from pam_partition_count. */
pam_status pam_partition_gather(pam_ctx *ctx, const pam_grid *grid, const double *cell_y,
                                const int64_t *off, double *x, double *y, double *h,
                                int32_t *cell);

/* ------------------------------------------------------------------------
 * Dictionary (Sec. 3.1: centers c_m and widths sigma_m; Alg. 1 input).
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_sub, dim, m_cap;
    int32_t *m;        /* [n_sub] current center counts (in/out)               */
    double *c;         /* [n_sub*m_cap*dim] centers                           */
    double *sigma;     /* [n_sub*m_cap] widths, > 0                           */
    int32_t *level;    /* [n_sub*m_cap] refinement level of each center       */
    int32_t basis;     /* PAM_BASIS_SHEPARD (default) or PAM_BASIS_PLAIN       */
} pam_dict;

/* Basis of the local expansion. SHEPARD: the normalized functions
 * phi_m / sum_k phi_k over the subdomain's whole dictionary (Sec. 3.2, Def. 1,
 * Eq. (shepard_rbf)), the method's own. PLAIN: the Gaussians phi_m
 * themselves, the unnormalized construction the paper compares against in
 * Example 1 (an ablation: every fit, indicator and evaluation entry point
 * then uses sum_m beta_m phi_m). */
enum { PAM_BASIS_SHEPARD = 0, PAM_BASIS_PLAIN = 1 };

/* a2. Initial dictionary: g[0]*..*g[dim-1] lattice at the cell centers of
 * each owned box, common width sigma0 = sigma_factor * max_axis(h_c) where
 * h_c = box width / g per axis (Exp. 1 "g x g lattice with width sigma").
 * g is [host]; requires product(g) <= m_cap. */
pam_status pam_init_lattice(pam_ctx *ctx, const pam_grid *grid, const int32_t *g,
                            double sigma_factor, pam_dict *dict);

/* ------------------------------------------------------------------------
 * Samples of every subdomain (Alg. 1 input: element sample points and the
 * data vector of log10 values).
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t dim, n_sub;
    int32_t n_max;            /* largest per-subdomain sample count            */
    const int64_t *off;       /* [n_sub+1] CSR offsets (device)                */
    const int64_t *off_host;  /* [host] same offsets                           */
    const double *x;          /* [N_tot*dim] sample points                     */
    const double *y;          /* [N_tot] data values (log10 K)                 */
    const double *h;          /* [N_tot*dim] element extents (indicator, enrichment) */
} pam_samples;

/* Elastic-net controls (Eq. elastic; lambda1, lambda2 > 0, optionally per
 * subdomain as the parallel implementation allows). */
typedef struct {
    double lambda1, lambda2;
    const double *lambda1_sub;   /* [n_sub] or NULL                            */
    const double *lambda2_sub;   /* [n_sub] or NULL                            */
    int32_t precision;           /* pam_precision                              */
    int32_t cd_sweeps;           /* cyclic CD warm-up sweeps (>= 0)            */
    int32_t max_iter;            /* active-set iteration cap (> 0)             */
    int32_t warm_start;          /* 1: beta holds the starting point           */
    int32_t batched;             /* 1: one launch per step for all subdomains;
                                    0: one launch per subdomain (comparator)   */
    const uint8_t *support_hint; /* [n_sub*m_cap] 1 = start active, or NULL.
                                    Used by cold fits only (warm_start = 0):
                                    replaces the CD warm-up by the hinted set
                                    S0, whose signs come from one FP64 ridge
                                    solve on S0; the exact iteration and KKT
                                    certificate follow, so beta is the same
                                    minimizer with or without a hint. In
                                    pam_refine it seeds the first fit only.  */
    int32_t team;                /* workgroups per subdomain in the solve of a
                                    batched launch: 0 = as many as fit on the
                                    device at once (4, else 2, else 1), 1 = one,
                                    2 or 4 = at most that many. A team's first
                                    workgroup runs the iteration; the others
                                    take row slices of its passes over the
                                    active-block inverse and the Gram. The
                                    minimizer and certificate are the same;
                                    sums are taken in another order. Unbatched
                                    launches always use one.                  */
    int32_t team_min;            /* active-set size from which a team shares
                                    those passes (0 = 128)                     */
    int32_t team_idle_us;        /* how long (us, <= 1e7) a team member waits
                                    for the next pass before it leaves (0 =
                                    10 s); the leader then does that member's
                                    rows itself, with the same result          */
} pam_enet_opts;

/* Per-subdomain results (device array of n_sub). */
typedef struct {
    int32_t status;     /* PAM_ST_*                                           */
    int32_t cd_sweeps;  /* CD sweeps done                                     */
    int32_t iters;      /* active-set iterations                              */
    int32_t support;    /* number of nonzero coefficients                     */
    double kkt;         /* KKT residual of the returned beta: max over m of
                           |g_m - lambda1 sign(beta_m)| (active) or
                           (|g_m| - lambda1)+ (inactive), g the FP64 gradient
                           of the smooth part (FP32/BF16 modes: from the FP64
                           design, not the rounded Gram)                     */
    double stream_bytes; /* bytes of Gram rows and active-block inverse the
                            solve had to stream (algorithmic traffic)        */
    int32_t polish;     /* FP32/BF16 Gram: FP64 conjugate-gradient steps of the
                           polish on the final support (negative: stopped
                           early on a sign change or lost curvature, the kkt
                           field then shows how far from the FP64 minimizer);
                           0 for FP64                                         */
    int32_t team;       /* workgroups that served the solve (1, 2 or 4)        */
    double solve_us;    /* wall time of this subdomain's solve on the device
                           (constant clock, microseconds), from its start to
                           its result: the per-subdomain cost of the batched
                           launch                                             */
} pam_fit_stats;

/* a3-a6. For every subdomain: Gaussian RBF design at the samples (Eq.
 * gaussian_rbf), Shepard row normalization W (Def. 1, Eq. shepard_rbf), normal
 * products G = W'W, b = W'y, and the unique elastic-net minimizer
 *   argmin 1/2||y - W beta||^2 + lambda1||beta||_1 + lambda2/2||beta||^2
 * (Eq. elastic, Sec. 3.3): CD warm-up, exact sign-consistent active-set
 * finish in FP64, KKT certificate. beta [n_sub*m_cap] (in: warm start if
 * opts->warm_start, out: coefficients; slots >= m[s] are set to 0).
 * stats: [n_sub] or NULL. */
pam_status pam_fit_subdomains(pam_ctx *ctx, const pam_samples *samples, const pam_dict *dict,
                              const pam_enet_opts *opts, double *beta, pam_fit_stats *stats);

/* a3-a6 again, with the FP64 Gram (PAM_PREC_F64) and from a cold start, for
 * exactly the subdomains whose stats entry reads PAM_ST_NOCONV: the recovery
 * for fits of the FP32/BF16 modes whose FP64 refinement reached its iteration
 * cap (the same minimizer, Eq. elastic, Sec. 3.3). samples, dict and beta as
 * in pam_fit_subdomains; stats [n_sub] (device, required) holds the previous
 * fit's entries on input. The refitted subdomains get new coefficients and
 * stats entries; every other subdomain's beta and stats stay as they were.
 * opts gives lambdas, cd_sweeps, max_iter, batched and the team settings; its
 * precision, warm_start and support_hint are ignored. Stream-ordered after
 * the fit that wrote stats (the mask is read on the device); the host waits
 * only when the FP64 workspace has to grow. Errors as pam_fit_subdomains
 * (the FP64 capacity limit applies to m_cap). */
pam_status pam_refit_nonconverged(pam_ctx *ctx, const pam_samples *samples, const pam_dict *dict,
                                  const pam_enet_opts *opts, double *beta, pam_fit_stats *stats);

/* Refinement controls (Alg. 1 inputs K_top, M_max, eps_tol; Sec. 3.4 eta). */
typedef struct {
    int32_t k_top;              /* elements marked per round                   */
    const int32_t *k_top_sub;   /* [host] per-subdomain K_top, or NULL          */
    int32_t max_rounds;         /* enrichment rounds after the first fit        */
    int32_t m_max;              /* max centers added per subdomain              */
    double eta;                 /* width factor of new centers, in (0, 1)      */
    double eps_tol;             /* stop when max R_T < eps_tol; only elements
                                   with R_T >= eps_tol are marked              */
    int32_t space;              /* 0: R_T on log10 values, 1: on 10^values     */
    int32_t *elem_level;        /* [N_tot] times each element was marked (in/out) */
    int32_t *rounds;            /* [n_sub] fits done per subdomain (out) or NULL */
    double *round_stats;        /* [n_sub*(max_rounds+1)*7] per round
                                   {M, support, max R_T, marked, sum R_T,
                                   solve stream bytes, solve wall time in us},
                                   or NULL                                     */
    int32_t cold_rounds;        /* 0: each refit starts from the previous beta
                                   extended by zeros (Alg. 1); 1: each refit
                                   starts from zero (comparator; same result,
                                   more work)                                  */
} pam_refine_opts;

/* a3-a9 (Alg. 1): fit, residual indicator R_T (Sec. 2 Step 3, 2-point
 * Gauss-Legendre per axis), stop test, marking of the K_top largest R_T,
 * enrichment with 2^dim-1 centers per marked element at
 * x_T + (h_T/2^(l+1)) o, o in {0,1}^dim \ {0}, widths sigma0*eta^(l+1)
 * (Sec. 3.4), zero-extension of beta and refit, for all subdomains at once.
 * dict is updated in place; requires m_cap >= m + m_max growth room or the
 * additions are truncated at m_cap. */
pam_status pam_refine(pam_ctx *ctx, const pam_samples *samples, pam_dict *dict, double *beta,
                      const pam_enet_opts *opts, const pam_refine_opts *ropts,
                      pam_fit_stats *stats);

/* ------------------------------------------------------------------------
 * a10. Global reconstruction (Sec. 2 Step 4): K*(x) = K*_{omega_i}(x) for x
 * in the owned box omega_i, with the local normalized expansion
 * sum_m beta_m phi_m(x) / sum_m phi_m(x) over the owner's whole dictionary.
 * Owners are found per axis from the owned breakpoints (half-open, last
 * interval closed). Points outside the closed domain give NaN.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t dim;
    int32_t n_sub_axis[3];
    const double *axis_x;   /* [host] per-axis owned breakpoint coordinates,
                               concatenated (n_sub_axis[a]+1 each)             */
    int32_t sub_base;       /* index of this field's first subdomain in dict  */
    int64_t q_begin, q_end; /* this field's query range                      */
} pam_field;

/* Evaluate n_fields fields (subdomains of all fields share dict/beta) at
 * their query ranges in one pass. dtype 0: xq is float [Q*dim] and out is
 * float [Q]; dtype 1: double. space 0: log10 values, 1: 10^values.
 * n_outside: device int64 counter of out-of-domain queries (added to), or
 * NULL. */
pam_status pam_eval(pam_ctx *ctx, int32_t n_fields, const pam_field *fields,
                    const pam_dict *dict, const double *beta, int32_t dtype, const void *xq,
                    int64_t Q, void *out, int32_t space, int64_t *n_outside);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): pam_eval with the same
 * arguments, result and kernels, allocating nothing. The binning workspace
 * is a fixed 64 MiB device array of the library (one per GPU, set up by
 * pam_create and held until the process ends) instead of the context's
 * workspace, and the field tables travel as a kernel argument instead of a
 * staged upload. Limits, checked on the host before anything is enqueued
 * (PAM_ERR_CAPACITY beyond them): n_fields <= 8, at most 240 breakpoints over
 * all fields and axes, and at most 64 MiB of binning workspace (about 12 B
 * per query plus 24 B per subdomain, 256-byte aligned pieces: up to about 5e6
 * queries per call). Kernel timing is not recorded. Every call on a GPU
 * shares that GPU's array and leaves its last contents there (each call
 * clears what it needs): calls that overlap in time on one GPU (other
 * streams, other threads) race, and the caller must order them. */
pam_status pam_eval_noalloc(pam_ctx *ctx, int32_t n_fields, const pam_field *fields,
                            const pam_dict *dict, const double *beta, int32_t dtype,
                            const void *xq, int64_t Q, void *out, int32_t space,
                            int64_t *n_outside);

/* ------------------------------------------------------------------------
 * Per-subdomain elastic-net parameters (Sec. 2 after Eq. (elastic): they may
 * differ between subdomains; Exp. 1.2 chooses them independently per
 * subdomain; the paper does not say how). lambda1 = l1_ratio * alpha,
 * lambda2 = (1 - l1_ratio) * alpha (l1_ratio = 0.99 reproduces the printed
 * pair 4.59e-4 / 4.64e-6 at alpha = 4.64e-4). alpha runs down the geometric
 * path alpha_k = alpha_max * alpha_min_ratio^(k / (n_alpha - 1)),
 * k = 0..n_alpha-1, from alpha_max = max_m |(W^T y)_m| / l1_ratio, the
 * smallest alpha at which the fit on all of the subdomain's samples is zero
 * (FP64, over the whole dictionary). Each alpha is scored by k_folds-fold
 * cross-validation: fold f of a subdomain holds its samples whose local index
 * j has j % k_folds == f; score = (1/N) sum_j (y_j - K*_f(x_j))^2, with K*_f
 * the surrogate fitted on the other folds (normalized over the whole
 * dictionary, FP64). The chosen alpha is the first (largest) with the
 * smallest score.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_alpha;        /* path length, 1..4096                           */
    int32_t k_folds;        /* 2..64                                          */
    double alpha_min_ratio; /* (0, 1]: last alpha / alpha_max                 */
    double l1_ratio;        /* (0, 1]: lambda1 / (lambda1 + lambda2)          */
} pam_select_opts;

/* Runs the path for all subdomains at once: the k_folds training sets of
 * every subdomain are fitted as one batch of n_sub * k_folds subdomains per
 * alpha (opts gives precision, cd_sweeps, max_iter, batched; its lambdas,
 * warm_start and support_hint are ignored), each warm-started from the
 * previous alpha's solution; the fits are the FP64 problem's minimizers in
 * every precision mode. Outputs (device, caller-owned): alpha and score
 * [n_sub * n_alpha] (row per subdomain), best [n_sub] (chosen index),
 * lambda1_sub / lambda2_sub [n_sub] (ready for pam_enet_opts), n_failed
 * [n_sub] or NULL (fits on the path whose status was neither OK nor EMPTY).
 * Workspace: the training sets, dictionaries and coefficients of the
 * n_sub * k_folds fits, from the context. Same argument checks as
 * pam_fit_subdomains plus the ranges above (PAM_ERR_ARG). */
pam_status pam_select_lambda(pam_ctx *ctx, const pam_samples *samples, const pam_dict *dict,
                             const pam_enet_opts *opts, const pam_select_opts *sel, double *alpha,
                             double *score, int32_t *best, double *lambda1_sub,
                             double *lambda2_sub, int32_t *n_failed);

/* ------------------------------------------------------------------------
 * Interface treatment (Sec. 2 Step 4 and the remark after it: the piecewise
 * K* of independent local fits is discontinuous across subdomain interfaces
 * in general; a continuous reconstruction averages neighbouring local
 * surrogates).
 *
 * Weights: a tensor-product partition of unity over the owned boxes. At an
 * interior breakpoint b_i of an axis, with neighbouring interval lengths
 * L_{i-1}, L_i, the band |t - b_i| < h_i, h_i = blend * min(L_{i-1}, L_i),
 * gives the interval on the left the weight 1 - rho(s) and the one on the
 * right rho(s), s = (t - b_i + h_i) / (2 h_i), rho(s) = s^2 (3 - 2 s) (C1);
 * outside the bands the owner interval has weight 1. The weight of a
 * subdomain is the product over the axes, and
 *   K_blend(x) = sum_i w_i(x) K*_i(x)
 * over the (at most 2^dim) subdomains with w_i(x) > 0, K*_i the local
 * normalized expansion over subdomain i's whole dictionary. The result is
 * continuous (C1 in the weights), equals the owner reconstruction
 * bit-for-bit outside the bands, and at an interface is the mean of the two
 * one-sided local surrogates. blend = 0 gives pam_eval's result exactly.
 * With a fit overlap delta > 0 (pam_grid.overlap), blend <= delta keeps every
 * surrogate inside the region it was fitted on.
 * ------------------------------------------------------------------------ */

/* Continuous reconstruction at the query points. Arguments as pam_eval, plus
 * blend in [0, 1/2] (PAM_ERR_ARG otherwise). Averaging is in log10 space;
 * space 1 exponentiates the averaged value. The per-query sum runs in a fixed
 * order, so results do not depend on the binning. Workspace: 2^dim slots of
 * the query type plus 2^dim int64 positions per query, from the context. */
pam_status pam_eval_blend(pam_ctx *ctx, int32_t n_fields, const pam_field *fields,
                          const pam_dict *dict, const double *beta, double blend, int32_t dtype,
                          const void *xq, int64_t Q, void *out, int32_t space,
                          int64_t *n_outside);

/* [host] Number of interior interface pieces of the fields' partitions:
 * sum over fields and axes a of (n_a - 1) * prod_{b != a} n_b; -1 on bad
 * arguments. No device work. */
int64_t pam_interface_count(int32_t n_fields, const pam_field *fields);

/* Jump of the piecewise reconstruction across every interior interface
 * piece, in FP64. Pieces are ordered by field, then axis a, then the upper
 * subdomain B (k_a >= 1) in linear order (axis 0 fastest); the lower one is
 * A = B - e_a. Each piece is sampled at the n_per_axis^(dim-1) midpoints of
 * a regular subdivision of B's face at b = B's lower breakpoint on axis a.
 * out: device double [2 * pam_interface_count], per piece
 * (max |K*_A - K*_B|, mean |K*_A - K*_B|). Query ranges of the fields are
 * ignored. n_per_axis in [1, 4096] and at most 2^24 samples per piece. */
pam_status pam_interface_jump(pam_ctx *ctx, int32_t n_fields, const pam_field *fields,
                              const pam_dict *dict, const double *beta, int32_t n_per_axis,
                              double *out);

/* ------------------------------------------------------------------------
 * Darcy consumer of the reconstruction (Sec. 5, Eq. (darcy_model); the
 * pressure experiment of Exp. 1): -div(K grad p) = 0 on the 2-D box
 * [lo, hi], p = p_left on the face x = lo[0], p = p_right on x = hi[0], no
 * flow across the other faces; continuous P1 finite elements on the
 * n[0] x n[1] squares of the box, each split along its diagonal from node
 * (i, j) to node (i+1, j+1) into a lower-right triangle (i,j),(i+1,j),
 * (i+1,j+1) and an upper-left one (i,j),(i+1,j+1),(i,j+1); nodes numbered
 * i + (n[0] + 1) j. K is constant per triangle and given by the caller, e.g.
 * 10^K* at the triangle centroids from pam_eval (space 1) or the data's own
 * cell values.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t n[2];          /* squares per axis, >= 1                           */
    double lo[2], hi[2];   /* the box, lo < hi                                 */
    double p_left, p_right;
    double tol;            /* stop at ||r|| <= tol ||b||, b the right-hand side
                              once the Dirichlet values are moved to it      */
    int32_t max_iter;      /* >= 1                                             */
    int32_t check_every;   /* iterations between host convergence checks, >= 1 */
} pam_darcy_opts;

/* Solves for the nodal pressure by Jacobi-preconditioned conjugate gradients
 * in FP64 (Dirichlet nodes eliminated). k_tri: device double
 * [n[1]][n[0]][2] (0 lower-right, 1 upper-left), K > 0. p: device double
 * [(n[0]+1)(n[1]+1)]; with warm = 1 its free-node values are the starting
 * point, else the start is linear between the two Dirichlet values; on
 * return the solution. iters, rel_res: [host] outputs (iterations taken and
 * the final ||r|| / ||b||; 0 when b = 0, whose solution is 0). Synchronizes the context's stream every
 * check_every iterations. Workspace: seven node vectors and the edge
 * weights, from the context. */
pam_status pam_darcy_solve(pam_ctx *ctx, const pam_darcy_opts *opts, const double *k_tri,
                           double *p, int32_t warm, int32_t *iters, double *rel_res);

/* Relative L2(Omega) error of two P1 pressures on the same mesh (Eq.
 * (pressure_L2_error)): ||p_ref - p|| / ||p_ref|| with the exact P1 mass
 * matrix (per triangle |T| / 12 (sum u_a^2 + (sum u_a)^2)), summed in FP64 in
 * a fixed order. p_ref, p: device double [(n[0]+1)(n[1]+1)]; e_rel: [host]
 * output (0 if ||p_ref|| = 0). Synchronizes the context's stream. */
pam_status pam_darcy_error(pam_ctx *ctx, const pam_darcy_opts *opts, const double *p_ref,
                           const double *p, double *e_rel);

/* Coefficient of the pressure problem from the reconstruction (Sec. 5: the
 * permeability of Eq. (darcy_model) is the surrogate K* of the fitted field;
 * the experiment of Exp. 1 solves with it on the mesh): k_tri
 * [n[1]][n[0]][2] (triangle order as above) = 10^K* at the centroid of every
 * triangle of the mesh of opts, K* the field's owner reconstruction (blend <
 * 0, as pam_eval) or its continuous reconstruction with band blend in
 * [0, 1/2] (as pam_eval_blend), in FP64. field: one 2-D field (its query
 * range is ignored). Workspace: the 2 n[0] n[1] centroids and the
 * evaluation's own, from the context. */
pam_status pam_darcy_coefficient(pam_ctx *ctx, const pam_darcy_opts *opts, const pam_field *field,
                                 const pam_dict *dict, const double *beta, double blend,
                                 double *k_tri);

/* The data's own coefficient on a mesh whose squares are the data cells:
 * both triangles of square (i, j) get 10^cell_y[i + n[0] j] (cell_y: device
 * double [n[0] n[1]], log10 values, axis 0 fastest). The reference pressure
 * of the relative error of Exp. 1 is solved with it. */
pam_status pam_darcy_coefficient_cells(pam_ctx *ctx, const pam_darcy_opts *opts,
                                       const double *cell_y, double *k_tri);

/* ------------------------------------------------------------------------
 * Learned warm start (not part of the paper's method: a support prior for
 * the cold elastic-net fits). A four-layer convolutional network, 5x5
 * "same" convolutions with zero padding, 1 -> 32 -> 32 -> 32 -> 2 channels,
 * ReLU after the first three, on 16x16 patches of cell values. Output
 * channel 0: per-cell refinement logit (target: the cell is marked in the
 * first refinement round); channel 1: per-cell support logit (target: the
 * center lying in the cell is active in the cold fit).
 *
 * Parameters: float [pam_cnn_param_count()] = 53,698, FP32, per layer
 * w[cout][cin][5][5] followed by b[cout], layers in order. Patches float
 * [B][1][16][16], logits and targets float [B][2][16][16], row-major with the
 * cell's axis-0 index fastest. All device pointers, caller-owned.
 * ------------------------------------------------------------------------ */
int64_t pam_cnn_param_count(void);

/* logits = network(params, x) for B >= 1 patches. precision: PAM_PREC_F32
 * (every layer on the vector ALUs in FP32) or PAM_PREC_BF16 (the two 32 -> 32
 * layers on BF16 MFMA with FP32 accumulation, activations and the thin first
 * and last layers in FP32); other values are rejected. */
pam_status pam_cnn_forward(pam_ctx *ctx, const float *params, int32_t B, const float *x,
                           float *logits, int32_t precision);

/* Masked binary cross-entropy with logits over both channels (precision as
 * for pam_cnn_forward; BF16 also runs the 32 -> 32 layers' backward-data and
 * weight-gradient products on MFMA),
 *   L = sum mask * (max(z,0) - z*t + log(1 + exp(-|z|))) / sum mask,
 * and its gradient with respect to every parameter (grads, same layout as
 * params, overwritten). loss: device float scalar or NULL. A batch with an
 * all-zero mask gives L = 0 and zero gradients. */
pam_status pam_cnn_loss_grad(pam_ctx *ctx, const float *params, int32_t B, const float *x,
                             const float *target, const float *mask, float *grads, float *loss,
                             int32_t precision);

/* One Adam step (Kingma and Ba, 2015) with bias correction at step >= 1:
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps). m, v: device
 * float [param_count] moment buffers, zero before step 1. */
pam_status pam_cnn_adam(pam_ctx *ctx, float *params, const float *grads, float *m, float *v,
                        int32_t step, float lr, float beta1, float beta2, float eps);

/* Cut the owned box of every subdomain of a 2-D grid (its sides must be
 * positive multiples of 16 cells) into 16x16 patches, numbered by
 * subdomain, then row-major over the patch grid (axis 0 fastest); patch
 * value = scale * cell_y. cell_y: device double [n_cells0*n_cells1] with
 * axis 0 fastest. *n_patches [host] receives the count; patches == NULL
 * makes this a count query. */
pam_status pam_grid_patches(pam_ctx *ctx, const pam_grid *grid, const double *cell_y, float scale,
                            int32_t *n_patches, float *patches);

/* Support hint from the network's logits over the patches of the same grid
 * (pam_grid_patches order): center k < m[s] of subdomain s reads the cell
 * containing it (floor of its cell coordinate, clamped into the owned box)
 * and is hinted active when that cell's support logit exceeds threshold
 * (0 = probability 1/2). hint: device uint8 [n_sub*m_cap]; slots >= m[s]
 * are set to 0. */
pam_status pam_support_hint(pam_ctx *ctx, const pam_grid *grid, const pam_dict *dict,
                            const float *logits, float threshold, uint8_t *hint);

/* Training targets and masks [n_patches][2][16][16] from the method's own
 * results on the same grid (the dictionary and samples of its partition):
 * support channel: cells holding a center (located as in pam_support_hint)
 * get mask 1 and target 1 iff a center in the cell has beta != 0 (beta: the
 * cold fit); refinement channel: owned cells of the samples get mask 1 and
 * target 1 iff elem_level > 0 (after one refinement round). Everything else
 * gets mask 0, target 0. */
pam_status pam_cnn_labels(pam_ctx *ctx, const pam_grid *grid, const pam_samples *samples,
                          const pam_dict *dict, const double *beta, const int32_t *elem_level,
                          float *target, float *mask);

/* ------------------------------------------------------------------------
 * Kernel timing (observability). When enabled, every kernel launch of the
 * context is bracketed by HIP events on the context's stream.
 * pam_timing_read synchronizes the stream and returns, per kernel kind, the
 * summed device time in milliseconds and the number of launches since the
 * last reset; reset = 1 clears the totals afterwards. EVAL_BIN covers the
 * query (or term) binning passes of both reconstructions and the weighted
 * sum of the continuous one; EVAL and BLEND the evaluation of the binned
 * queries and terms; JUMP the interface-jump kernel; DARCY a whole Darcy solve.
 * ------------------------------------------------------------------------ */
enum {
    PAM_TK_GATHER = 0, PAM_TK_LATTICE, PAM_TK_ASSEMBLE, PAM_TK_GRAM, PAM_TK_SOLVE,
    PAM_TK_INDICATOR, PAM_TK_MARK, PAM_TK_EVAL_BIN, PAM_TK_EVAL, PAM_TK_CNN,
    PAM_TK_BLEND, PAM_TK_JUMP, PAM_TK_DARCY, PAM_TK_COUNT
};
pam_status pam_timing_enable(pam_ctx *ctx, int32_t on);
pam_status pam_timing_read(pam_ctx *ctx, double *ms /*[host] PAM_TK_COUNT*/,
                           int64_t *launches /*[host] PAM_TK_COUNT*/, int32_t reset);

#ifdef __cplusplus
}
#endif
#endif /* PAM_H */
