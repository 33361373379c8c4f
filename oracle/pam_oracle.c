/*
 * PAM reconstruction oracle: a plain, slow, FP64 CPU implementation of the
 * per-subdomain path of the Parallel and Adaptive Mesh-free method (PAM).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library calls, links or
 * includes this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it. It shares no code, header, table or
 * constant with the HIP library.
 *
 * Every loop is written in the order the paper states the step, in FP64,
 * with no blocking or fusion. Compiled with -ffp-contract=off so that the
 * handful of expressions that must be bit-reproducible (sample centroids,
 * lattice centers, enriched centers) round exactly once per operation.
 *
 * Sections of the paper followed (cited per function):
 *   Sec. 2 Step 1      domain decomposition into half-open subdomains
 *   Sec. 2 Step 2      samples at element centroids, data vector, feature matrix
 *   Sec. 3.1 Eq. (gaussian_rbf)          Gaussian RBF
 *   Sec. 3.2 Def. 1, Eq. (shepard_rbf)   Shepard normalization
 *   Sec. 2 Eq. (elastic), Sec. 3.3       elastic net, coordinate descent
 *   Sec. 2 Step 3, Alg. 1 (2)            residual indicator R_T
 *   Alg. 1 (3), until-test               marking and stopping
 *   Sec. 3.4, Alg. 1 (4)-(5)             enrichment, dictionary update
 *   Sec. 2 Step 4                        global reconstruction / evaluation
 *   Eq. (L2error)                        relative L2 error metric
 *   Sec. 2 after Eq. (elastic), Exp. 1.2 per-subdomain choice of the elastic-
 *                                        net parameters (path + cross-validation)
 *   Sec. 2 Step 4, Remark after it       interface treatment: averaging of
 *                                        neighbouring local surrogates and
 *                                        the jump of the piecewise K* across
 *                                        subdomain interfaces
 *
 * Readings where the paper is silent (all documented with the design notes):
 *   - the regression is on the Shepard-normalized matrix W, and the surrogate
 *     is the normalized expansion over the whole dictionary;
 *   - data are log10 values, objective uses the literal 1/2 scaling, no
 *     intercept, no column standardization;
 *   - the elastic-net result is the unique minimizer (lambda2 > 0): cyclic CD
 *     warm-up, then an exact sign-consistent active-set finish (feature-sign
 *     search) and a KKT certificate;
 *   - R_T uses 2-point Gauss-Legendre per axis, weights |T|/2^d, in log10
 *     space by default (linear space optional);
 *   - stop test after R_T and before enrichment; marked elements are the
 *     K_top largest R_T (ties by element index) among those with R_T >= tol;
 *   - enrichment adds, per marked element T at level l, the 2^d-1 centers
 *     x_T + (h_T / 2^(l+1)) * o, o in {0,1}^d \ {0}, width sigma0 * eta^(l+1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>

#define ORA_OK 0
#define ORA_ERR_ARG (-1)
#define ORA_ERR_CAPACITY (-2)
#define ORA_ERR_UNDERFLOW (-4)
#define ORA_NOCONV 1

/* ------------------------------------------------------------------------- */
/* a1. Partition of a structured grid and sample gathering                   */
/* Sec. 2 Step 1 (non-overlapping half-open subdomains, each element in one   */
/* subdomain, Exp. 1.2) and Step 2 (one sample per element at its centroid,   */
/* data vector of cell values). Optional overlap widens only the fit set.    */
/* ------------------------------------------------------------------------- */

/* Cell-index range [first, last) along one axis whose centroids i+1/2 lie in
 * the fit interval of subdomain k: the owned interval [b_k, b_{k+1}) widened
 * by overlap*(b_{k+1}-b_k) on interior faces only. */
static void ora_axis_range(int n_cells, int n_sub, const int *breaks, int k,
                           double overlap, int *first, int *last)
{
    double b0 = (double)breaks[k], b1 = (double)breaks[k + 1];
    double w = b1 - b0;
    double lo = b0, hi = b1;
    if (k > 0) lo = b0 - overlap * w;
    if (k < n_sub - 1) hi = b1 + overlap * w;
    int f = -1, l = -1;
    for (int i = 0; i < n_cells; ++i) {
        double u = (double)i + 0.5;
        if (u >= lo && u < hi) {
            if (f < 0) f = i;
            l = i + 1;
        }
    }
    if (f < 0) { f = 0; l = 0; }
    *first = f;
    *last = l;
}

/* Sample counts per subdomain (row-major over subdomains, axis 0 fastest).
 * off has n_sub_total+1 entries. Returns total sample count or <0. */
long ora_partition_count(int dim, const int *n_cells, const int *n_sub,
                         const int *breaks_flat, double overlap, long *off)
{
    if (dim < 1 || dim > 3 || overlap < 0.0) return ORA_ERR_ARG;
    const int *brk[3];
    int pos = 0;
    int ns[3] = {1, 1, 1};
    for (int a = 0; a < dim; ++a) {
        ns[a] = n_sub[a];
        brk[a] = breaks_flat + pos;
        pos += n_sub[a] + 1;
    }
    long total = 0;
    long s = 0;
    off[0] = 0;
    for (int k2 = 0; k2 < ns[2]; ++k2)
        for (int k1 = 0; k1 < ns[1]; ++k1)
            for (int k0 = 0; k0 < ns[0]; ++k0) {
                int kk[3] = {k0, k1, k2};
                long cnt = 1;
                for (int a = 0; a < dim; ++a) {
                    int f, l;
                    ora_axis_range(n_cells[a], n_sub[a], brk[a], kk[a], overlap, &f, &l);
                    cnt *= (long)(l - f);
                }
                total += cnt;
                off[++s] = total;
            }
    return total;
}

/* Gather the samples: centroid x_T = lo + (i+1/2) h, value y_T, extents h_T,
 * integer cell index per axis. Cells of a subdomain are listed row-major
 * (axis 0 fastest), subdomains likewise. */
int ora_partition_gather(int dim, const int *n_cells, const double *dom_lo,
                         const double *dom_hi, const int *n_sub,
                         const int *breaks_flat, double overlap,
                         const double *cell_y, const long *off, double *x,
                         double *y, double *h, int *cell)
{
    const int *brk[3];
    int pos = 0;
    int ns[3] = {1, 1, 1};
    int nc[3] = {1, 1, 1};
    double hh[3] = {1, 1, 1};
    for (int a = 0; a < dim; ++a) {
        ns[a] = n_sub[a];
        nc[a] = n_cells[a];
        brk[a] = breaks_flat + pos;
        pos += n_sub[a] + 1;
        hh[a] = (dom_hi[a] - dom_lo[a]) / (double)n_cells[a];
    }
    long s = 0;
    for (int k2 = 0; k2 < ns[2]; ++k2)
        for (int k1 = 0; k1 < ns[1]; ++k1)
            for (int k0 = 0; k0 < ns[0]; ++k0) {
                int kk[3] = {k0, k1, k2};
                int f[3] = {0, 0, 0}, l[3] = {1, 1, 1};
                for (int a = 0; a < dim; ++a)
                    ora_axis_range(n_cells[a], n_sub[a], brk[a], kk[a], overlap, &f[a], &l[a]);
                long j = off[s];
                for (int i2 = f[2]; i2 < l[2]; ++i2)
                    for (int i1 = f[1]; i1 < l[1]; ++i1)
                        for (int i0 = f[0]; i0 < l[0]; ++i0) {
                            int ii[3] = {i0, i1, i2};
                            long g = (long)i0 + (long)nc[0] * ((long)i1 + (long)nc[1] * (long)i2);
                            for (int a = 0; a < dim; ++a) {
                                x[j * dim + a] = dom_lo[a] + ((double)ii[a] + 0.5) * hh[a];
                                h[j * dim + a] = hh[a];
                                cell[j * dim + a] = ii[a];
                            }
                            y[j] = cell_y[g];
                            ++j;
                        }
                if (j != off[s + 1]) return ORA_ERR_ARG;
                ++s;
            }
    return ORA_OK;
}

/* ------------------------------------------------------------------------- */
/* a2. Initial dictionary: uniform g^d lattice at cell centers of the owned   */
/* box, common width sigma0 (Sec. 1, Exp. 1 "g x g lattice with width").      */
/* sigma0 = sigma_factor * max_axis(h_c).                                     */
/* ------------------------------------------------------------------------- */
int ora_lattice(int dim, const double *box_lo, const double *box_hi,
                const int *g, double sigma_factor, double *c, double *sigma,
                int *level)
{
    int gg[3] = {1, 1, 1};
    double hc[3] = {0, 0, 0};
    double hmax = 0.0;
    for (int a = 0; a < dim; ++a) {
        gg[a] = g[a];
        hc[a] = (box_hi[a] - box_lo[a]) / (double)g[a];
        if (hc[a] > hmax) hmax = hc[a];
    }
    double s0 = sigma_factor * hmax;
    int m = 0;
    for (int j2 = 0; j2 < gg[2]; ++j2)
        for (int j1 = 0; j1 < gg[1]; ++j1)
            for (int j0 = 0; j0 < gg[0]; ++j0) {
                int jj[3] = {j0, j1, j2};
                for (int a = 0; a < dim; ++a)
                    c[m * dim + a] = box_lo[a] + ((double)jj[a] + 0.5) * hc[a];
                sigma[m] = s0;
                level[m] = 0;
                ++m;
            }
    return m;
}

/* ------------------------------------------------------------------------- */
/* a3 + a4. Gaussian RBF (Eq. gaussian_rbf) and Shepard-normalized design     */
/* W_jm = phi_m(x_j) / sum_k phi_k(x_j) (Def. 1, Eq. shepard_rbf).            */
/* ------------------------------------------------------------------------- */
static double ora_phi(int dim, const double *x, const double *c, double sigma)
{
    double r2 = 0.0;
    for (int a = 0; a < dim; ++a) {
        double d = x[a] - c[a];
        r2 += d * d;
    }
    return exp(-r2 / (2.0 * sigma * sigma));
}

/* Basis of the local expansion, a process-wide switch that the Python
 * wrappers set before every call: 0 = Shepard-normalized (Sec. 3.2, the
 * method's), 1 = the plain Gaussians (the unnormalized comparison of
 * Example 1). Every function below builds its design with ora_design and
 * evaluates with ora_surrogate, the only two places that read it. */
static int ora_plain = 0;

void ora_set_basis(int plain) { ora_plain = plain ? 1 : 0; }

/* W is N x M row-major. Returns ORA_ERR_UNDERFLOW if a row sum is not a
 * positive normal number (the normalization is defined only where the sum of
 * the basis functions is positive). The plain basis keeps phi itself. */
int ora_design(int dim, int N, int M, const double *x, const double *c,
               const double *sigma, double *W)
{
    for (int j = 0; j < N; ++j) {
        double s = 0.0;
        for (int m = 0; m < M; ++m) {
            double p = ora_phi(dim, x + (long)j * dim, c + (long)m * dim, sigma[m]);
            W[(long)j * M + m] = p;
            s += p;
        }
        if (ora_plain) continue;
        if (!(s >= DBL_MIN)) return ORA_ERR_UNDERFLOW;
        for (int m = 0; m < M; ++m) W[(long)j * M + m] /= s;
    }
    return ORA_OK;
}

/* a5. Normal products G = W^T W (M x M), b = W^T y. Each entry is one plain
 * sum over the samples in index order; the transpose copy only makes the
 * sums read contiguous memory. */
void ora_normal(int N, int M, const double *W, const double *y, double *G,
                double *b)
{
    double *Wt = (double *)malloc(sizeof(double) * (size_t)N * (size_t)M + 8);
    for (int j = 0; j < N; ++j)
        for (int m = 0; m < M; ++m) Wt[(long)m * N + j] = W[(long)j * M + m];
#pragma omp parallel for schedule(dynamic, 8)
    for (int m = 0; m < M; ++m) {
        const double *wm = Wt + (long)m * N;
        for (int k = 0; k < M; ++k) {
            const double *wk = Wt + (long)k * N;
            double s = 0.0;
            for (int j = 0; j < N; ++j) s += wm[j] * wk[j];
            G[(long)m * M + k] = s;
        }
        double t = 0.0;
        for (int j = 0; j < N; ++j) t += wm[j] * y[j];
        b[m] = t;
    }
    free(Wt);
}

/* ------------------------------------------------------------------------- */
/* a6. Elastic net (Eq. elastic): minimize                                    */
/*   1/2 ||y - W beta||^2 + lambda1 ||beta||_1 + lambda2/2 ||beta||^2         */
/* written on the normal products: 1/2 b'Ab - b'beta + lambda1||beta||_1 with  */
/* A = G + lambda2 I. The minimizer is unique for lambda2 > 0.                */
/* ------------------------------------------------------------------------- */
static double ora_sign(double v) { return v > 0.0 ? 1.0 : (v < 0.0 ? -1.0 : 0.0); }

/* Cyclic coordinate descent sweeps in creation order (Sec. 3.3), covariance
 * form with gradient g = b - A beta maintained. Returns sweeps done. */
int ora_cd(int M, const double *G, const double *b, double lambda1,
           double lambda2, int max_sweeps, double tol, double *beta)
{
    double *g = (double *)malloc(sizeof(double) * (size_t)(M > 0 ? M : 1));
    for (int m = 0; m < M; ++m) {
        double s = b[m];
        for (int k = 0; k < M; ++k) s -= G[(long)m * M + k] * beta[k];
        g[m] = s - lambda2 * beta[m];
    }
    int sw = 0;
    while (sw < max_sweeps) {
        ++sw;
        double dmax = 0.0, bmax = 0.0;
        for (int m = 0; m < M; ++m) {
            double gmm = G[(long)m * M + m];
            double z = g[m] + (gmm + lambda2) * beta[m];
            double az = fabs(z) - lambda1;
            double nb = az > 0.0 ? ora_sign(z) * az / (gmm + lambda2) : 0.0;
            double d = nb - beta[m];
            if (d != 0.0) {
                for (int k = 0; k < M; ++k) g[k] -= G[(long)k * M + m] * d;
                g[m] -= lambda2 * d;
                beta[m] = nb;
                if (fabs(d) > dmax) dmax = fabs(d);
            }
            if (fabs(beta[m]) > bmax) bmax = fabs(beta[m]);
        }
        if (dmax <= tol * (bmax > 1.0 ? bmax : 1.0)) break;
    }
    free(g);
    return sw;
}

/* Solve (A_SS) z = r by Cholesky (A SPD), with 2 steps of iterative
 * refinement. A is M x M (full, includes lambda2 on the diagonal), S lists s
 * indices. Returns 0 or -1 if A_SS is not numerically positive definite. */
static int ora_solve_sub(int M, const double *A, const int *S, int s,
                         const double *r, double *z)
{
    double *L = (double *)malloc(sizeof(double) * (size_t)s * (size_t)s + 8);
    double *t = (double *)malloc(sizeof(double) * (size_t)s + 8);
    double *e = (double *)malloc(sizeof(double) * (size_t)s + 8);
    for (int i = 0; i < s; ++i)
        for (int j = 0; j <= i; ++j) {
            double v = A[(long)S[i] * M + S[j]];
            for (int k = 0; k < j; ++k) v -= L[(long)i * s + k] * L[(long)j * s + k];
            if (i == j) {
                if (!(v > 0.0)) { free(L); free(t); free(e); return -1; }
                L[(long)i * s + i] = sqrt(v);
            } else {
                L[(long)i * s + j] = v / L[(long)j * s + j];
            }
        }
    /* z = L^-T L^-1 r, then refine with the residual of A_SS. */
    for (int i = 0; i < s; ++i) e[i] = r[i];
    for (int i = 0; i < s; ++i) z[i] = 0.0;
    for (int pass = 0; pass < 3; ++pass) {
        for (int i = 0; i < s; ++i) {
            double v = e[i];
            for (int k = 0; k < i; ++k) v -= L[(long)i * s + k] * t[k];
            t[i] = v / L[(long)i * s + i];
        }
        for (int i = s - 1; i >= 0; --i) {
            double v = t[i];
            for (int k = i + 1; k < s; ++k) v -= L[(long)k * s + i] * t[k];
            t[i] = v / L[(long)i * s + i];
        }
        for (int i = 0; i < s; ++i) z[i] += t[i];
        for (int i = 0; i < s; ++i) {
            double v = r[i];
            for (int k = 0; k < s; ++k) v -= A[(long)S[i] * M + S[k]] * z[k];
            e[i] = v;
        }
    }
    free(L);
    free(t);
    free(e);
    return 0;
}

/* Objective difference f(beta0 + t d) - f(beta0) on the support S, where
 * c1 = (A_SS beta0 - b_S) . d and c2 = d' A_SS d. */
static double ora_seg_obj(int s, const double *b0, const double *d, double t,
                          double c1, double c2, double lambda1)
{
    double l1 = 0.0;
    for (int i = 0; i < s; ++i) l1 += fabs(b0[i] + t * d[i]) - fabs(b0[i]);
    return t * c1 + 0.5 * t * t * c2 + lambda1 * l1;
}

/* Exact finish: sign-consistent active-set iteration (feature-sign search of
 * Lee, Battle, Raina and Ng, 2007), adapted to the elastic net. Starting from
 * beta (any warm start), it alternates (i) the equality-constrained solve on
 * the current signed support followed by a discrete line search over the
 * zero crossings, and (ii) activation of the inactive coordinate with the
 * largest KKT violation. The objective decreases strictly, so the loop ends
 * at the unique minimizer. Returns iterations or -1 (no convergence). */
int ora_fss(int M, const double *G, const double *b, double lambda1,
            double lambda2, int max_iter, double kkt_tol, double *beta)
{
    double *A = (double *)malloc(sizeof(double) * (size_t)M * (size_t)M + 8);
    for (long i = 0; i < (long)M * M; ++i) A[i] = G[i];
    for (int m = 0; m < M; ++m) A[(long)m * M + m] += lambda2;
    double *th = (double *)malloc(sizeof(double) * (size_t)M + 8);
    int *S = (int *)malloc(sizeof(int) * (size_t)M + 8);
    double *r = (double *)malloc(sizeof(double) * (size_t)M + 8);
    double *z = (double *)malloc(sizeof(double) * (size_t)M + 8);
    double *b0 = (double *)malloc(sizeof(double) * (size_t)M + 8);
    double *d = (double *)malloc(sizeof(double) * (size_t)M + 8);
    double *g = (double *)malloc(sizeof(double) * (size_t)M + 8);
    double bnorm = 0.0;
    for (int m = 0; m < M; ++m) {
        th[m] = ora_sign(beta[m]);
        if (fabs(b[m]) > bnorm) bnorm = fabs(b[m]);
    }
    int it = 0, ret = -1;
    while (it < max_iter) {
        ++it;
        int s = 0;
        for (int m = 0; m < M; ++m)
            if (th[m] != 0.0) S[s++] = m;
        if (s > 0) {
            for (int i = 0; i < s; ++i) r[i] = b[S[i]] - lambda1 * th[S[i]];
            if (ora_solve_sub(M, A, S, s, r, z) != 0) break;
            int consistent = 1;
            for (int i = 0; i < s; ++i)
                if (ora_sign(z[i]) != th[S[i]]) consistent = 0;
            if (!consistent) {
                /* discrete line search from the current point to z */
                for (int i = 0; i < s; ++i) {
                    b0[i] = beta[S[i]];
                    d[i] = z[i] - b0[i];
                }
                double c1 = 0.0, c2 = 0.0;
                for (int i = 0; i < s; ++i) {
                    double ab = 0.0, ad = 0.0;
                    for (int k = 0; k < s; ++k) {
                        ab += A[(long)S[i] * M + S[k]] * b0[k];
                        ad += A[(long)S[i] * M + S[k]] * d[k];
                    }
                    c1 += (ab - b[S[i]]) * d[i];
                    c2 += d[i] * ad;
                }
                double best_t = 1.0;
                double best_f = ora_seg_obj(s, b0, d, 1.0, c1, c2, lambda1);
                for (int i = 0; i < s; ++i) {
                    if (b0[i] != 0.0 && ora_sign(z[i]) != ora_sign(b0[i])) {
                        double t = b0[i] / (b0[i] - z[i]);
                        if (t > 0.0 && t < 1.0) {
                            double f = ora_seg_obj(s, b0, d, t, c1, c2, lambda1);
                            if (f < best_f) { best_f = f; best_t = t; }
                        }
                    }
                }
                for (int i = 0; i < s; ++i) {
                    double v = b0[i] + best_t * d[i];
                    if (best_t < 1.0 && b0[i] != 0.0 && ora_sign(z[i]) != ora_sign(b0[i])) {
                        double t = b0[i] / (b0[i] - z[i]);
                        if (t == best_t) v = 0.0;
                    }
                    beta[S[i]] = v;
                }
                for (int m = 0; m < M; ++m) th[m] = ora_sign(beta[m]);
                continue;
            }
            for (int i = 0; i < s; ++i) beta[S[i]] = z[i];
        }
        for (int m = 0; m < M; ++m)
            if (th[m] == 0.0) beta[m] = 0.0;
        /* KKT on inactive coordinates: |b - A beta| <= lambda1 */
        int kmax = -1;
        double vmax = 0.0;
        for (int m = 0; m < M; ++m) {
            double v = b[m];
            for (int k = 0; k < M; ++k) v -= A[(long)m * M + k] * beta[k];
            g[m] = v;
            if (beta[m] == 0.0 && fabs(v) > vmax) { vmax = fabs(v); kmax = m; }
        }
        if (kmax < 0 || vmax <= lambda1 * (1.0 + kkt_tol) + 1e-14 * bnorm) {
            ret = it;
            break;
        }
        th[kmax] = ora_sign(g[kmax]);
    }
    free(A); free(th); free(S); free(r); free(z); free(b0); free(d); free(g);
    return ret;
}

/* KKT residual of beta: active coordinates |g_m - lambda1 sign(beta_m)|,
 * inactive max(|g_m| - lambda1, 0), with g = b - (G + lambda2 I) beta. */
double ora_kkt(int M, const double *G, const double *b, double lambda1,
               double lambda2, const double *beta)
{
    double worst = 0.0;
    for (int m = 0; m < M; ++m) {
        double v = b[m] - lambda2 * beta[m];
        for (int k = 0; k < M; ++k) v -= G[(long)m * M + k] * beta[k];
        double e = beta[m] != 0.0 ? fabs(v - lambda1 * ora_sign(beta[m]))
                                  : (fabs(v) > lambda1 ? fabs(v) - lambda1 : 0.0);
        if (e > worst) worst = e;
    }
    return worst;
}

/* a3-a6 for one subdomain. beta (length M) holds the warm start on entry
 * (zeros for a cold start, Alg. 1 initialization; zero-extended previous
 * coefficients after enrichment, Alg. 1 (5)). Returns status; sweeps/iters
 * and the KKT residual are written to stats[0..2]. */
int ora_fit_one(int dim, int N, int M, const double *x, const double *y,
                const double *c, const double *sigma, double lambda1,
                double lambda2, int cd_sweeps, double *beta, double *stats)
{
    double *W = (double *)malloc(sizeof(double) * (size_t)N * (size_t)M + 8);
    double *G = (double *)malloc(sizeof(double) * (size_t)M * (size_t)M + 8);
    double *b = (double *)malloc(sizeof(double) * (size_t)M + 8);
    int st = ora_design(dim, N, M, x, c, sigma, W);
    if (st != ORA_OK) {
        free(W); free(G); free(b);
        return st;
    }
    ora_normal(N, M, W, y, G, b);
    int sw = ora_cd(M, G, b, lambda1, lambda2, cd_sweeps, 1e-13, beta);
    int it = ora_fss(M, G, b, lambda1, lambda2, 100000, 1e-12, beta);
    double kkt = ora_kkt(M, G, b, lambda1, lambda2, beta);
    if (stats) {
        stats[0] = sw;
        stats[1] = it;
        stats[2] = kkt;
    }
    free(W); free(G); free(b);
    return it < 0 ? ORA_NOCONV : ORA_OK;
}

/* ------------------------------------------------------------------------- */
/* a10. Local surrogate (normalized expansion, Sec. 3.2) at one point.        */
/* ------------------------------------------------------------------------- */
static double ora_surrogate(int dim, int M, const double *c, const double *sigma,
                            const double *beta, const double *xq)
{
    double num = 0.0, den = 0.0;
    for (int m = 0; m < M; ++m) {
        double p = ora_phi(dim, xq, c + (long)m * dim, sigma[m]);
        num += beta[m] * p;
        den += p;
    }
    return ora_plain ? num : num / den;
}

/* ------------------------------------------------------------------------- */
/* a7. Residual indicator R_T (Sec. 2 Step 3, Alg. 1 (2)): 2-point Gauss-     */
/* Legendre per axis at x_T +- h_T/(2 sqrt 3), weights |T|/2^d.               */
/* space 0: log10 values; space 1: 10^(.) of both (Alg. 1 literal).            */
/* ------------------------------------------------------------------------- */
void ora_indicator(int dim, int N, int M, const double *x, const double *y,
                   const double *h, const double *c, const double *sigma,
                   const double *beta, int space, double *R)
{
    int nq = 1 << dim;
    double off = 1.0 / (2.0 * sqrt(3.0));
    for (int j = 0; j < N; ++j) {
        double vol = 1.0;
        for (int a = 0; a < dim; ++a) vol *= h[(long)j * dim + a];
        double w = vol / (double)nq;
        double acc = 0.0;
        for (int q = 0; q < nq; ++q) {
            double xq[3];
            for (int a = 0; a < dim; ++a) {
                double sgn = ((q >> a) & 1) ? 1.0 : -1.0;
                xq[a] = x[(long)j * dim + a] + sgn * off * h[(long)j * dim + a];
            }
            double v = ora_surrogate(dim, M, c, sigma, beta, xq);
            double e = space == 0 ? v - y[j] : pow(10.0, v) - pow(10.0, y[j]);
            acc += w * e * e;
        }
        R[j] = acc;
    }
}

/* a8. Marking (Alg. 1 (3)): indices of the (up to) k_top largest R_T with
 * R_T >= tol, ranked by R descending then index ascending. Returns count. */
int ora_mark(int N, const double *R, int k_top, double tol, int *marked)
{
    int cnt = 0;
    char *used = (char *)calloc((size_t)N + 1, 1);
    while (cnt < k_top) {
        int best = -1;
        for (int j = 0; j < N; ++j) {
            if (used[j] || !(R[j] >= tol)) continue;
            if (best < 0 || R[j] > R[best]) best = j;
        }
        if (best < 0) break;
        used[best] = 1;
        marked[cnt++] = best;
    }
    free(used);
    return cnt;
}

/* a9. Enrichment (Sec. 3.4, Alg. 1 (4)-(5)): for each marked element in rank
 * order, append 2^d - 1 centers at x_T + (h_T * 2^-(l+1)) * o, o in {0,1}^d
 * without 0 (o = bits of q = 1 .. 2^d-1, axis 0 lowest), widths
 * sigma0 * eta^(l+1), level l+1; l = times T was marked before. Stops before
 * an element whose whole group does not fit under m_limit. Returns new M. */
int ora_enrich(int dim, int M, int m_limit, const double *x, const double *h,
               int n_marked, const int *marked, double sigma0, double eta,
               int *elem_level, double *c, double *sigma, int *level)
{
    int per = (1 << dim) - 1;
    for (int r = 0; r < n_marked; ++r) {
        if (M + per > m_limit) break;
        int j = marked[r];
        int l = elem_level[j];
        double scale = 1.0;
        for (int i = 0; i <= l; ++i) scale *= 0.5;
        double sw = sigma0;
        for (int i = 0; i <= l; ++i) sw *= eta;
        for (int q = 1; q <= per; ++q) {
            for (int a = 0; a < dim; ++a) {
                double o = (double)((q >> a) & 1);
                c[(long)M * dim + a] = x[(long)j * dim + a] + (h[(long)j * dim + a] * scale) * o;
            }
            sigma[M] = sw;
            level[M] = l + 1;
            ++M;
        }
        elem_level[j] = l + 1;
    }
    return M;
}

/* ------------------------------------------------------------------------- */
/* Alg. 1 for one subdomain: fit, indicator, stop/mark, enrich, refit.        */
/* Dictionary arrays have capacity m_cap; m (in/out) is the count; beta is    */
/* length m_cap (warm start in, result out). round_stats[r*5 + 0..3] =        */
/* {M, support, max R, marked} per round. Returns status; *rounds_out =       */
/* number of fits done. round_stats[r*5 + 4] = sum of R_T (the squared       */
/* L2 error of the fit set under the indicator's quadrature).                 */
/* ------------------------------------------------------------------------- */
int ora_refine_one(int dim, int N, const double *x, const double *y,
                   const double *h, int m_cap, int *m, double *c,
                   double *sigma, int *level, double *beta, int *elem_level,
                   double lambda1, double lambda2, int cd_sweeps, int k_top,
                   int max_rounds, int m_max, double eps_tol, double eta,
                   int space, double *round_stats, int *rounds_out)
{
    int M0 = *m;
    int limit = M0 + m_max;
    if (limit > m_cap) limit = m_cap;
    double sigma0 = sigma[0];
    double *R = (double *)malloc(sizeof(double) * (size_t)N + 8);
    int *marked = (int *)malloc(sizeof(int) * (size_t)N + 8);
    int status = ORA_OK;
    int r = 0;
    for (;;) {
        double st[3];
        status = ora_fit_one(dim, N, *m, x, y, c, sigma, lambda1, lambda2, cd_sweeps, beta, st);
        int supp = 0;
        for (int k = 0; k < *m; ++k) supp += beta[k] != 0.0;
        ora_indicator(dim, N, *m, x, y, h, c, sigma, beta, space, R);
        double rmax = 0.0, rsum = 0.0;
        for (int j = 0; j < N; ++j) {
            if (R[j] > rmax) rmax = R[j];
            rsum += R[j];
        }
        int nm = 0;
        int stop = status != ORA_OK || rmax < eps_tol || r >= max_rounds || *m >= limit;
        if (!stop) nm = ora_mark(N, R, k_top, eps_tol, marked);
        if (round_stats) {
            round_stats[r * 5 + 0] = *m;
            round_stats[r * 5 + 1] = supp;
            round_stats[r * 5 + 2] = rmax;
            round_stats[r * 5 + 3] = nm;
            round_stats[r * 5 + 4] = rsum;
        }
        ++r;
        if (stop || nm == 0) break;
        int m_new = ora_enrich(dim, *m, limit, x, h, nm, marked, sigma0, eta, elem_level, c, sigma, level);
        if (m_new == *m) break;
        for (int k = *m; k < m_new; ++k) beta[k] = 0.0;
        *m = m_new;
    }
    *rounds_out = r;
    free(R);
    free(marked);
    return status;
}

/* Batched drivers over subdomains (OpenMP over subdomains when compiled with
 * it; the per-subdomain work is the plain code above). Dictionary layout:
 * c[s*m_cap*dim], sigma[s*m_cap], level[s*m_cap], beta[s*m_cap], m[s].     */
int ora_fit_batch(int dim, int n_sub, const long *off, const double *x,
                  const double *y, int m_cap, const int *m, const double *c,
                  const double *sigma, double lambda1, double lambda2,
                  int cd_sweeps, double *beta, double *stats, int *status)
{
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad) if (n_sub > 1)
    for (int s = 0; s < n_sub; ++s) {
        long j0 = off[s];
        int N = (int)(off[s + 1] - j0);
        status[s] = ora_fit_one(dim, N, m[s], x + j0 * dim, y + j0,
                                c + (long)s * m_cap * dim, sigma + (long)s * m_cap,
                                lambda1, lambda2, cd_sweeps,
                                beta + (long)s * m_cap, stats ? stats + 3L * s : 0);
        bad += status[s] != ORA_OK;
    }
    return bad;
}

int ora_refine_batch(int dim, int n_sub, const long *off, const double *x,
                     const double *y, const double *h, int m_cap, int *m,
                     double *c, double *sigma, int *level, double *beta,
                     int *elem_level, double lambda1, double lambda2,
                     int cd_sweeps, const int *k_top, int max_rounds, int m_max,
                     double eps_tol, double eta, int space, double *round_stats,
                     int *rounds, int *status)
{
    int bad = 0;
    int rs = max_rounds + 1;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad) if (n_sub > 1)
    for (int s = 0; s < n_sub; ++s) {
        long j0 = off[s];
        int N = (int)(off[s + 1] - j0);
        status[s] = ora_refine_one(
            dim, N, x + j0 * dim, y + j0, h + j0 * dim, m_cap, m + s,
            c + (long)s * m_cap * dim, sigma + (long)s * m_cap,
            level + (long)s * m_cap, beta + (long)s * m_cap, elem_level + j0,
            lambda1, lambda2, cd_sweeps, k_top[s], max_rounds, m_max, eps_tol, eta,
            space, round_stats ? round_stats + (long)s * rs * 5 : 0, rounds + s);
        bad += status[s] != ORA_OK;
    }
    return bad;
}

/* ------------------------------------------------------------------------- */
/* a10. Global reconstruction and evaluation (Sec. 2 Step 4): the owner       */
/* subdomain of x is found per axis from the owned breakpoints (half-open,    */
/* last interval closed); K*(x) is the owner's normalized expansion. Points   */
/* outside the closed domain give NaN. space 1 returns 10^value.             */
/* axis_x: per-axis breakpoint coordinates, concatenated (n_sub[a]+1 each).  */
/* Returns the number of points outside the domain.                          */
/* ------------------------------------------------------------------------- */
long ora_eval(int dim, const int *n_sub, const double *axis_x, int m_cap,
              const int *m, const double *c, const double *sigma,
              const double *beta, long Q, const double *xq, int space,
              double *out)
{
    long outside = 0;
#pragma omp parallel for schedule(static) reduction(+ : outside)
    for (long q = 0; q < Q; ++q) {
        int pos = 0, sub = 0, stride = 1, ok = 1;
        for (int a = 0; a < dim; ++a) {
            const double *bx = axis_x + pos;
            int n = n_sub[a];
            double v = xq[q * dim + a];
            if (!(v >= bx[0] && v <= bx[n])) { ok = 0; break; }
            int k = n - 1;
            for (int i = 0; i < n; ++i)
                if (v < bx[i + 1]) { k = i; break; }
            sub += k * stride;
            stride *= n;
            pos += n + 1;
        }
        if (!ok) {
            out[q] = NAN;
            ++outside;
            continue;
        }
        double v = ora_surrogate(dim, m[sub], c + (long)sub * m_cap * dim,
                                 sigma + (long)sub * m_cap,
                                 beta + (long)sub * m_cap, xq + q * dim);
        out[q] = space == 1 ? pow(10.0, v) : v;
    }
    return outside;
}

/* ------------------------------------------------------------------------- */
/* Interface treatment (Sec. 2 Step 4 and the remark after it: the piecewise  */
/* K* is discontinuous across subdomain interfaces in general; a continuous  */
/* reconstruction averages neighbouring local surrogates).                   */
/*                                                                           */
/* Reading (the paper names the idea, not the weights): a tensor-product     */
/* partition of unity over the subdomain boxes. On each axis, interval j of  */
/* the owned breakpoints b_0 < ... < b_n has the weight                      */
/*   omega_j(t) = rho((t - b_j + h_j) / (2 h_j))                on the left  */
/*                                                 band |t - b_j| < h_j,     */
/*   omega_j(t) = 1 - rho((t - b_{j+1} + h_{j+1}) / (2 h_{j+1})) on the right */
/*                                                 band |t - b_{j+1}| < h_{j+1},*/
/*   1 between the bands and 0 outside [b_j - h_j, b_{j+1} + h_{j+1}],        */
/* with band half-width h_i = blend * min(L_{i-1}, L_i) at an interior        */
/* breakpoint (L = interval lengths), h = 0 at the domain ends, and the C1    */
/* ramp rho(s) = s^2 (3 - 2 s) on [0, 1]. With h = 0 the weight is the        */
/* half-open indicator of the owned interval (last one closed), so blend = 0  */
/* gives the owner reconstruction. The blended field is                       */
/*   K_blend(x) = sum_i w_i(x) K*_i(x),  w_i = prod_a omega_{i_a}(x_a),       */
/* summed over every subdomain i (zero weights skipped), K*_i the local       */
/* normalized expansion. Requires 0 <= blend <= 1/2 (bands of one interval    */
/* do not overlap).                                                           */
/* ------------------------------------------------------------------------- */
static double ora_rho(double s)
{
    if (s <= 0.0) return 0.0;
    if (s >= 1.0) return 1.0;
    return s * s * (3.0 - 2.0 * s);
}

static double ora_band(const double *bx, int n, int i, double blend)
{
    if (i <= 0 || i >= n) return 0.0;
    return blend * fmin(bx[i] - bx[i - 1], bx[i + 1] - bx[i]);
}

static double ora_interval_weight(const double *bx, int n, int j, double blend, double t)
{
    double w = 1.0;
    double hl = ora_band(bx, n, j, blend), hr = ora_band(bx, n, j + 1, blend);
    if (j > 0) {
        if (hl > 0.0) {
            if (t <= bx[j] - hl) return 0.0;
            if (t < bx[j] + hl) w = ora_rho((t - (bx[j] - hl)) / (2.0 * hl));
        } else if (t < bx[j]) {
            return 0.0;
        }
    }
    if (j < n - 1) {
        if (hr > 0.0) {
            if (t >= bx[j + 1] + hr) return 0.0;
            if (t > bx[j + 1] - hr) w = 1.0 - ora_rho((t - (bx[j + 1] - hr)) / (2.0 * hr));
        } else if (t >= bx[j + 1]) {
            return 0.0;
        }
    }
    return w;
}

long ora_eval_blend(int dim, const int *n_sub, const double *axis_x, double blend, int m_cap,
                    const int *m, const double *c, const double *sigma, const double *beta,
                    long Q, const double *xq, int space, double *out)
{
    long outside = 0;
    int n_tot = 1, off[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) {
        n_tot *= n_sub[a];
        if (a > 0) off[a] = off[a - 1] + n_sub[a - 1] + 1;
    }
#pragma omp parallel for schedule(static) reduction(+ : outside)
    for (long q = 0; q < Q; ++q) {
        const double *x = xq + q * dim;
        int inside = 1;
        for (int a = 0; a < dim; ++a) {
            const double *bx = axis_x + off[a];
            if (!(x[a] >= bx[0] && x[a] <= bx[n_sub[a]])) inside = 0;
        }
        if (!inside) {
            out[q] = NAN;
            ++outside;
            continue;
        }
        double acc = 0.0;
        for (int i = 0; i < n_tot; ++i) {
            double w = 1.0;
            int rest = i;
            for (int a = 0; a < dim; ++a) {
                int k = rest % n_sub[a];
                rest /= n_sub[a];
                w *= ora_interval_weight(axis_x + off[a], n_sub[a], k, blend, x[a]);
            }
            if (w == 0.0) continue;
            acc += w * ora_surrogate(dim, m[i], c + (long)i * m_cap * dim, sigma + (long)i * m_cap,
                                     beta + (long)i * m_cap, x);
        }
        out[q] = space == 1 ? pow(10.0, acc) : acc;
    }
    return outside;
}

/* Jump of the piecewise K* across every interior interface piece: for axis  */
/* a and each subdomain B with index k_a >= 1 (linear order, axis 0 fastest), */
/* the face shared with A = B - e_a, sampled at the n^(dim-1) midpoints of a  */
/* regular n-per-axis subdivision of the face; out[2f] = max |K*_A - K*_B|,  */
/* out[2f+1] = mean |K*_A - K*_B| over the samples. Faces ordered by axis,    */
/* then B. Returns the number of faces.                                       */
long ora_interface_jump(int dim, const int *n_sub, const double *axis_x, int m_cap, const int *m,
                        const double *c, const double *sigma, const double *beta, int n,
                        double *out)
{
    int ns[3] = {1, 1, 1}, off[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) {
        ns[a] = n_sub[a];
        if (a > 0) off[a] = off[a - 1] + n_sub[a - 1] + 1;
    }
    int n_tot = ns[0] * ns[1] * ns[2];
    long f = 0;
    for (int a = 0; a < dim; ++a) {
        for (int B = 0; B < n_tot; ++B) {
            int kk[3] = {B % ns[0], (B / ns[0]) % ns[1], B / (ns[0] * ns[1])};
            if (kk[a] == 0) continue;
            int stride = a == 0 ? 1 : (a == 1 ? ns[0] : ns[0] * ns[1]);
            int A = B - stride;
            int n_pts = 1;
            for (int b = 0; b < dim - 1; ++b) n_pts *= n;
            double mx = 0.0, sum = 0.0;
            for (int p = 0; p < n_pts; ++p) {
                double x[3];
                int rest = p;
                for (int b = 0; b < dim; ++b) {
                    const double *bx = axis_x + off[b];
                    if (b == a) {
                        x[b] = bx[kk[b]];
                    } else {
                        int j = rest % n;
                        rest /= n;
                        double lo = bx[kk[b]], hi = bx[kk[b] + 1];
                        x[b] = lo + (j + 0.5) * (hi - lo) / n;
                    }
                }
                double vA = ora_surrogate(dim, m[A], c + (long)A * m_cap * dim,
                                          sigma + (long)A * m_cap, beta + (long)A * m_cap, x);
                double vB = ora_surrogate(dim, m[B], c + (long)B * m_cap * dim,
                                          sigma + (long)B * m_cap, beta + (long)B * m_cap, x);
                double j = fabs(vA - vB);
                if (j > mx) mx = j;
                sum += j;
            }
            out[2 * f] = mx;
            out[2 * f + 1] = sum / n_pts;
            ++f;
        }
    }
    return f;
}

/* ------------------------------------------------------------------------- */
/* Per-subdomain choice of the elastic-net parameters (Sec. 2 after Eq.      */
/* (elastic): they may differ between subdomains; Exp. 1.2: chosen           */
/* independently per subdomain). The paper does not say how; reading:        */
/*   lambda1 = rho * alpha, lambda2 = (1 - rho) * alpha with a fixed mixing   */
/*   rho (0.99 reproduces the printed pair 4.59e-4 / 4.64e-6);               */
/*   alpha on a geometric grid of n_alpha values from                         */
/*   alpha_max = max_m |(W^T y)_m| / rho, the smallest alpha at which the fit */
/*   on all the subdomain's samples is zero, down to alpha_max * ratio;       */
/*   K-fold cross-validation, fold(j) = j mod K on the subdomain's local      */
/*   sample index; score(alpha) = (1/N) sum over folds of the squared errors  */
/*   of the held-out samples under the fit on the other folds;                */
/*   chosen: the first (largest) alpha with the smallest score.              */
/* Every fit is an independent cold fit (ora_fit_one).                        */
/* alpha, score: [n_sub * n_alpha]; best: [n_sub]. Returns the number of     */
/* failed fits.                                                               */
/* ------------------------------------------------------------------------- */
int ora_select_lambda(int dim, int n_sub, const long *off, const double *x, const double *y,
                      int m_cap, const int *m, const double *c, const double *sigma,
                      int n_alpha, double ratio, double rho, int k_folds, int cd_sweeps,
                      double *alpha, double *score, int *best)
{
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
    for (int s = 0; s < n_sub; ++s) {
        const long j0 = off[s];
        const int N = (int)(off[s + 1] - j0), M = m[s];
        const double *xs = x + j0 * dim, *ys = y + j0;
        const double *cs = c + (long)s * m_cap * dim, *sg = sigma + (long)s * m_cap;
        double *W = (double *)malloc(sizeof(double) * ((size_t)N * M + 1));
        double *xt = (double *)malloc(sizeof(double) * ((size_t)N * dim + 1));
        double *yt = (double *)malloc(sizeof(double) * ((size_t)N + 1));
        double *beta = (double *)malloc(sizeof(double) * ((size_t)M + 1));
        double st3[3];
        double amax = 0.0;
        if (ora_design(dim, N, M, xs, cs, sg, W) != ORA_OK) {
            ++bad;
        } else {
            for (int mm = 0; mm < M; ++mm) {
                double bm = 0.0;
                for (int j = 0; j < N; ++j) bm += W[(long)j * M + mm] * ys[j];
                if (fabs(bm) > amax) amax = fabs(bm);
            }
            amax /= rho;
        }
        for (int k = 0; k < n_alpha; ++k) {
            double a = n_alpha > 1 ? amax * pow(ratio, (double)k / (double)(n_alpha - 1)) : amax;
            alpha[(long)s * n_alpha + k] = a;
            double err = 0.0;
            for (int f = 0; f < k_folds; ++f) {
                int nt = 0;
                for (int j = 0; j < N; ++j) {
                    if (j % k_folds == f) continue;
                    for (int d = 0; d < dim; ++d) xt[(long)nt * dim + d] = xs[(long)j * dim + d];
                    yt[nt++] = ys[j];
                }
                for (int mm = 0; mm < M; ++mm) beta[mm] = 0.0;
                if (ora_fit_one(dim, nt, M, xt, yt, cs, sg, rho * a, (1.0 - rho) * a, cd_sweeps,
                                beta, st3) != ORA_OK)
                    ++bad;
                for (int j = f; j < N; j += k_folds) {
                    double e = ys[j] - ora_surrogate(dim, M, cs, sg, beta, xs + (long)j * dim);
                    err += e * e;
                }
            }
            score[(long)s * n_alpha + k] = N > 0 ? err / N : 0.0;
        }
        int kb = 0;
        for (int k = 1; k < n_alpha; ++k)
            if (score[(long)s * n_alpha + k] < score[(long)s * n_alpha + kb]) kb = k;
        best[s] = kb;
        free(W); free(xt); free(yt); free(beta);
    }
    return bad;
}
