// Per-subdomain choice of the elastic-net parameters (Sec. 2 after Eq.
// (elastic): the parameters may differ between subdomains; Exp. 1.2 chooses
// them independently per subdomain). lambda1 = rho alpha, lambda2 =
// (1 - rho) alpha; alpha runs down a geometric path from the full-data zero
// threshold alpha_max = max_m |(W^T y)_m| / rho; each alpha is scored by
// K-fold cross-validation (fold of a sample = its local index mod K).
//
// The K training sets of every subdomain become K "virtual subdomains"
// (same dictionary, the other folds' samples), so every path step is one
// batched fit of n_sub * K subdomains through the ordinary fit kernels, warm
// started from the previous step. These kernels only build the virtual
// problem, the path, the held-out scores and the choice.
#include <float.h>

#include "pam_internal.h"

namespace pam {

static constexpr int kS = 256;     // threads per block
static constexpr int kSC = 512;    // centers staged in LDS per pass

// Virtual subdomain v = s * K + f keeps the samples j of s with j % K != f,
// in order: sample j lands at j - (number of held-out samples before j).
__global__ void __launch_bounds__(kS)
k_cv_gather(int n_sub, int K, int dim, const int64_t *__restrict__ off,
            const double *__restrict__ x, const double *__restrict__ y,
            const int64_t *__restrict__ off_v, double *__restrict__ xv, double *__restrict__ yv) {
    const int v = blockIdx.x;
    if (v >= n_sub * K) return;
    const int s = v / K, f = v % K;
    const int64_t j0 = off[s];
    const int N = (int)(off[s + 1] - j0);
    const int64_t o = off_v[v];
    for (int j = threadIdx.x; j < N; j += kS) {
        if (j % K == f) continue;
        const int held = j > f ? (j - 1 - f) / K + 1 : 0;
        const int64_t t = o + (j - held);
        for (int d = 0; d < dim; ++d) xv[t * dim + d] = x[(j0 + j) * dim + d];
        yv[t] = y[j0 + j];
    }
}

// Dictionary of every virtual subdomain: a copy of its subdomain's.
__global__ void __launch_bounds__(kS)
k_cv_dict(int n_sub, int K, int dim, int m_cap, const int32_t *__restrict__ m,
          const double *__restrict__ c, const double *__restrict__ sigma,
          const int32_t *__restrict__ level, int32_t *__restrict__ mv, double *__restrict__ cv,
          double *__restrict__ sv, int32_t *__restrict__ lv, double *__restrict__ beta_v) {
    const int v = blockIdx.x;
    if (v >= n_sub * K) return;
    const int s = v / K;
    if (threadIdx.x == 0) mv[v] = m[s];
    for (int i = threadIdx.x; i < m_cap * dim; i += kS)
        cv[(size_t)v * m_cap * dim + i] = c[(size_t)s * m_cap * dim + i];
    for (int i = threadIdx.x; i < m_cap; i += kS) {
        sv[(size_t)v * m_cap + i] = sigma[(size_t)s * m_cap + i];
        lv[(size_t)v * m_cap + i] = level[(size_t)s * m_cap + i];
        beta_v[(size_t)v * m_cap + i] = 0.0;
    }
}

__device__ __forceinline__ double block_sum(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int k = kS / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_max(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int k = kS / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + k]);
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// alpha path of subdomain s in FP64: row sums of the Gaussian design over the
// whole dictionary (inv_s = 1 / row sum), b_m = sum_j W_jm y_j, alpha_max =
// max |b| / rho, alpha_k = alpha_max * ratio^(k / (n_alpha - 1)).
__global__ void __launch_bounds__(kS)
k_alpha_path(int n_sub, int dim, int m_cap, const int64_t *__restrict__ off,
             const double *__restrict__ x, const double *__restrict__ y,
             const int32_t *__restrict__ m, const double *__restrict__ c,
             const double *__restrict__ sigma, double *__restrict__ inv_s, int n_alpha,
             double ratio, double rho, double *__restrict__ alpha, int plain) {
    const int s = blockIdx.x;
    if (s >= n_sub) return;
    __shared__ double red[kS];
    const int64_t j0 = off[s];
    const int N = (int)(off[s + 1] - j0);
    const int M = max(0, min(m[s], m_cap));
    const double *cs = c + (size_t)s * m_cap * dim;
    const double *sg = sigma + (size_t)s * m_cap;
    for (int j = threadIdx.x; j < N; j += kS) {
        double sum = 0.0;
        for (int mm = 0; mm < M; ++mm) {
            double r2 = 0.0;
            for (int d = 0; d < dim; ++d) {
                const double df = x[(j0 + j) * dim + d] - cs[(size_t)mm * dim + d];
                r2 += df * df;
            }
            sum += exp(-r2 / (2.0 * sg[mm] * sg[mm]));
        }
        inv_s[j0 + j] = plain ? 1.0 : (sum > 0.0 ? 1.0 / sum : 0.0);
    }
    __syncthreads();
    double amax = 0.0;
    for (int mm = threadIdx.x; mm < M; mm += kS) {
        double b = 0.0;
        const double a = 1.0 / (2.0 * sg[mm] * sg[mm]);
        for (int j = 0; j < N; ++j) {
            double r2 = 0.0;
            for (int d = 0; d < dim; ++d) {
                const double df = x[(j0 + j) * dim + d] - cs[(size_t)mm * dim + d];
                r2 += df * df;
            }
            b += exp(-r2 * a) * inv_s[j0 + j] * y[j0 + j];
        }
        amax = fmax(amax, fabs(b));
    }
    amax = block_max(amax, red) / rho;
    for (int k = threadIdx.x; k < n_alpha; k += kS)
        alpha[(size_t)s * n_alpha + k] =
            n_alpha > 1 ? amax * pow(ratio, (double)k / (double)(n_alpha - 1)) : amax;
}

// Parameters of path step k for every virtual subdomain.
__global__ void __launch_bounds__(kS)
k_cv_lambda(int n_sub, int K, int n_alpha, int k, double rho, const double *__restrict__ alpha,
            double *__restrict__ l1v, double *__restrict__ l2v) {
    const int v = blockIdx.x * kS + threadIdx.x;
    if (v >= n_sub * K) return;
    const double a = alpha[(size_t)(v / K) * n_alpha + k];
    l1v[v] = rho * a;
    l2v[v] = (1.0 - rho) * a;
}

// Held-out score of path step k for subdomain s (FP64): every sample j is
// predicted by the fit of fold j % K (the one that did not see it); the
// squared errors are summed in a fixed order, score = sum / N. Failed virtual
// fits (status != 0) are counted into n_failed[s].
__global__ void __launch_bounds__(kS)
k_cv_score(int n_sub, int K, int dim, int m_cap, int n_alpha, int k,
           const int64_t *__restrict__ off, const double *__restrict__ x,
           const double *__restrict__ y, const int32_t *__restrict__ m,
           const double *__restrict__ c, const double *__restrict__ sigma,
           const double *__restrict__ beta_v, const pam_fit_stats *__restrict__ stats_v,
           double *__restrict__ score, int32_t *__restrict__ n_failed, int plain) {
    const int s = blockIdx.x;
    if (s >= n_sub) return;
    __shared__ double sc[kSC * 3];
    __shared__ double sa[kSC];
    __shared__ double red[kS];
    const int64_t j0 = off[s];
    const int N = (int)(off[s + 1] - j0);
    const int M = max(0, min(m[s], m_cap));
    const double *cs = c + (size_t)s * m_cap * dim;
    const double *sg = sigma + (size_t)s * m_cap;
    double err = 0.0;
    for (int jb = 0; jb < N; jb += kS) {
        const int j = jb + threadIdx.x;
        const bool live = j < N;
        double xj[3] = {0.0, 0.0, 0.0};
        const double *bv = beta_v;
        if (live) {
            for (int d = 0; d < dim; ++d) xj[d] = x[(j0 + j) * dim + d];
            bv = beta_v + ((size_t)s * K + j % K) * m_cap;
        }
        double num = 0.0, den = 0.0;
        for (int m0 = 0; m0 < M; m0 += kSC) {
            const int cnt = min(kSC, M - m0);
            __syncthreads();
            for (int t = threadIdx.x; t < cnt; t += kS) {
                for (int d = 0; d < dim; ++d) sc[t * 3 + d] = cs[(size_t)(m0 + t) * dim + d];
                const double g = sg[m0 + t];
                sa[t] = 0.5 / (g * g);
            }
            __syncthreads();
            if (live) {
                for (int t = 0; t < cnt; ++t) {
                    double r2 = 0.0;
                    for (int d = 0; d < dim; ++d) {
                        const double df = xj[d] - sc[t * 3 + d];
                        r2 += df * df;
                    }
                    const double p = exp(-r2 * sa[t]);
                    num += bv[m0 + t] * p;
                    den += p;
                }
            }
        }
        if (live) {
            const double e = y[j0 + j] - (plain ? num : (den > 0.0 ? num / den : 0.0));
            err += e * e;
        }
    }
    err = block_sum(err, red);
    if (threadIdx.x == 0) {
        score[(size_t)s * n_alpha + k] = N > 0 ? err / N : 0.0;
        int bad = 0;
        for (int f = 0; f < K; ++f) bad += stats_v[(size_t)s * K + f].status != PAM_ST_OK &&
                                          stats_v[(size_t)s * K + f].status != PAM_ST_EMPTY;
        if (n_failed) n_failed[s] += bad;
    }
}

// Choice per subdomain: the first (largest) alpha with the smallest score.
__global__ void __launch_bounds__(kS)
k_cv_choose(int n_sub, int n_alpha, double rho, const double *__restrict__ alpha,
            const double *__restrict__ score, int32_t *__restrict__ best,
            double *__restrict__ l1, double *__restrict__ l2) {
    const int s = blockIdx.x * kS + threadIdx.x;
    if (s >= n_sub) return;
    int kb = 0;
    for (int k = 1; k < n_alpha; ++k)
        if (score[(size_t)s * n_alpha + k] < score[(size_t)s * n_alpha + kb]) kb = k;
    best[s] = kb;
    const double a = alpha[(size_t)s * n_alpha + kb];
    l1[s] = rho * a;
    l2[s] = (1.0 - rho) * a;
}

__global__ void __launch_bounds__(kS)
k_cv_zero(int n, int32_t *__restrict__ p) {
    const int i = blockIdx.x * kS + threadIdx.x;
    if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------- launchers
pam_status launch_cv_setup(pam_ctx *ctx, const pam_samples *S, const pam_dict *D, int K,
                           const int64_t *off_v, double *xv, double *yv, int32_t *mv, double *cv,
                           double *sv, int32_t *lv, double *beta_v, double *inv_s, int n_alpha,
                           double ratio, double rho, double *alpha, int32_t *n_failed) {
    const int n = S->n_sub, nv = n * K;
    hipLaunchKernelGGL(k_cv_gather, dim3(nv), dim3(kS), 0, ctx->stream, n, K, S->dim, S->off, S->x,
                       S->y, off_v, xv, yv);
    PAM_CHECK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_cv_dict, dim3(nv), dim3(kS), 0, ctx->stream, n, K, S->dim, D->m_cap, D->m,
                       D->c, D->sigma, D->level, mv, cv, sv, lv, beta_v);
    PAM_CHECK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_alpha_path, dim3(n), dim3(kS), 0, ctx->stream, n, S->dim, D->m_cap, S->off,
                       S->x, S->y, D->m, D->c, D->sigma, inv_s, n_alpha, ratio, rho, alpha,
                       D->basis == PAM_BASIS_PLAIN);
    PAM_CHECK_HIP(hipGetLastError());
    if (n_failed) {
        hipLaunchKernelGGL(k_cv_zero, dim3((n + kS - 1) / kS), dim3(kS), 0, ctx->stream, n, n_failed);
        PAM_CHECK_HIP(hipGetLastError());
    }
    return PAM_OK;
}

pam_status launch_cv_lambda(pam_ctx *ctx, int n_sub, int K, int n_alpha, int k, double rho,
                            const double *alpha, double *l1v, double *l2v) {
    hipLaunchKernelGGL(k_cv_lambda, dim3((n_sub * K + kS - 1) / kS), dim3(kS), 0, ctx->stream, n_sub,
                       K, n_alpha, k, rho, alpha, l1v, l2v);
    PAM_CHECK_HIP(hipGetLastError());
    return PAM_OK;
}

pam_status launch_cv_score(pam_ctx *ctx, const pam_samples *S, const pam_dict *D, int K,
                           int n_alpha, int k, const double *beta_v, const pam_fit_stats *stats_v,
                           double *score, int32_t *n_failed) {
    hipLaunchKernelGGL(k_cv_score, dim3(S->n_sub), dim3(kS), 0, ctx->stream, S->n_sub, K, S->dim,
                       D->m_cap, n_alpha, k, S->off, S->x, S->y, D->m, D->c, D->sigma, beta_v,
                       stats_v, score, n_failed, D->basis == PAM_BASIS_PLAIN);
    PAM_CHECK_HIP(hipGetLastError());
    return PAM_OK;
}

pam_status launch_cv_choose(pam_ctx *ctx, int n_sub, int n_alpha, double rho, const double *alpha,
                            const double *score, int32_t *best, double *l1, double *l2) {
    hipLaunchKernelGGL(k_cv_choose, dim3((n_sub + kS - 1) / kS), dim3(kS), 0, ctx->stream, n_sub,
                       n_alpha, rho, alpha, score, best, l1, l2);
    PAM_CHECK_HIP(hipGetLastError());
    return PAM_OK;
}

}  // namespace pam
