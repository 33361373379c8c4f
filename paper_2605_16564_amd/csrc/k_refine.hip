// Residual-driven adaptivity kernels (gfx950): indicator R_T, stop test and
// marking of the K_top largest indicators, enrichment with narrower centers.
// Sec. 2 Step 3; Alg. 1 steps (2)-(5); Sec. 3.4 (new widths eta * sigma).
#include <float.h>

#include "pam_internal.h"

namespace pam {

static constexpr int kT = 256;
static constexpr int kIC = 256;  // centers staged per pass

// R_T for every sample element of the active subdomains: 2-point
// Gauss-Legendre per axis at x_T +- h_T/(2 sqrt 3), weights |T| / 2^d, of the
// squared misfit of the normalized expansion (log10 values, or 10^values).
// One thread per element; all 2^d points accumulate against each staged
// center, in FP64 so that marking decisions follow the exact indicator. The
// dimension is a template parameter, so the 2^d points' coordinates and sums
// stay in registers.
template <int DIM>
__global__ void __launch_bounds__(kT)
k_indicator(RefineArgs a, double *__restrict__ R) {
    constexpr int NQ = 1 << DIM;
    const int s = blockIdx.y;
    if (!a.active[s]) return;
    const int64_t j0 = a.off[s];
    const int N = (int)(a.off[s + 1] - j0);
    const int j = blockIdx.x * kT + threadIdx.x;
    if (a.flags[s] & 2) {   // non-finite input: no indicator
        if (j < N) R[j0 + j] = __builtin_nan("");
        return;
    }
    const int M = max(0, min(a.m[s], a.m_cap));
    __shared__ double sc[kIC * DIM];
    __shared__ double sa[kIC];
    __shared__ double sb[kIC];
    double xq[NQ][DIM];
    double num[NQ], den[NQ];
    const bool live = j < N;
    double vol = 1.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        num[q] = 0.0;
        den[q] = 0.0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) xq[q][d] = 0.0;
    }
    if (live) {
        const double off = 0.28867513459481287;  // 1 / (2 sqrt 3)
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            const double hd = a.h[(j0 + j) * DIM + d];
            const double xd = a.x[(j0 + j) * DIM + d];
#pragma unroll
            for (int q = 0; q < NQ; ++q) xq[q][d] = xd + (((q >> d) & 1) ? 1.0 : -1.0) * off * hd;
            vol *= hd;
        }
    }
    const double *cs = a.c + (size_t)s * a.m_cap * DIM;
    const double *ss = a.sigma + (size_t)s * a.m_cap;
    const double *bs = a.beta + (size_t)s * a.m_cap;
    for (int m0 = 0; m0 < M; m0 += kIC) {
        const int cnt = min(kIC, M - m0);
        __syncthreads();
        for (int t = threadIdx.x; t < cnt * DIM; t += kT) sc[t] = cs[(size_t)m0 * DIM + t];
        for (int t = threadIdx.x; t < cnt; t += kT) {
            const double sg = ss[m0 + t];
            sa[t] = 0.5 / (sg * sg);
            sb[t] = bs[m0 + t];
        }
        __syncthreads();
        if (live) {
            for (int t = 0; t < cnt; ++t) {
                const double ia = sa[t], bt = sb[t];
                double cc[DIM];
#pragma unroll
                for (int d = 0; d < DIM; ++d) cc[d] = sc[t * DIM + d];
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    double r2 = 0.0;
#pragma unroll
                    for (int d = 0; d < DIM; ++d) {
                        const double df = xq[q][d] - cc[d];
                        r2 += df * df;
                    }
                    const double p = exp(-r2 * ia);
                    num[q] += bt * p;
                    den[q] += p;
                }
            }
        }
    }
    if (!live) return;
    const double yv = a.y[j0 + j];
    const double w = vol / (double)NQ;
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double v = a.basis == PAM_BASIS_PLAIN ? num[q] : num[q] / den[q];
        const double e = a.space == 0 ? v - yv : exp10(v) - exp10(yv);
        acc += w * e * e;
    }
    R[j0 + j] = acc;
}

pam_status launch_indicator(pam_ctx *ctx, const RefineArgs &a) {
    dim3 grid((a.n_max + kT - 1) / kT, a.n_sub);
    auto kern = a.dim == 1 ? k_indicator<1> : a.dim == 2 ? k_indicator<2> : k_indicator<3>;
    hipLaunchKernelGGL(kern, grid, dim3(kT), 0, ctx->stream, a, wsp<double>(ctx, BUF_R));
    PAM_CHECK_HIP(hipGetLastError());
    return PAM_OK;
}

// ---------------------------------------------------------------- mark + enrich
// One block per active subdomain:
//  1. max and sum of R_T; stop test (max R_T < eps_tol, last round, or the
//     center budget M0 + M_max reached), checked after the indicator and
//     before any enrichment, so every output dictionary is a fitted one;
//  2. rank the elements by (R_T descending, element index ascending) with a
//     bitonic sort in LDS and keep the first K_top with R_T >= eps_tol;
//  3. for each kept element T (rank order) with level l: append the 2^d - 1
//     centers x_T + (h_T 2^-(l+1)) o, o in {0,1}^d \ {0} (bits of q, axis 0
//     lowest), widths sigma0 eta^(l+1), level l + 1; a group that does not fit
//     under the budget ends the enrichment; beta is zero-extended.
// Up to kSortMax samples per subdomain the ranking runs in LDS; larger
// subdomains (up to kSortMaxGlobal) rank in a per-subdomain scratch area in
// HBM (BUF_MARK: P keys and P indices, P = n_max rounded up to a power of
// two) with the same sort.
static constexpr int kSortMax = 4096;
static constexpr int kSortMaxGlobal = 1 << 22;

__host__ __device__ inline int sort_len(int n) {
    int P = 1;
    while (P < n) P <<= 1;
    return P;
}

template <bool kGlobal>
__global__ void __launch_bounds__(kT)
k_mark_enrich(RefineArgs a, const double *__restrict__ R, char *__restrict__ sort_ws) {
#pragma clang fp contract(off)
    const int s = blockIdx.x;
    if (!a.active[s]) return;
    const int64_t j0 = a.off[s];
    const int N = (int)(a.off[s + 1] - j0);
    const int M = max(0, min(a.m[s], a.m_cap));
    const int dim = a.dim;
    __shared__ double key_l[kGlobal ? 1 : kSortMax];
    __shared__ int idx_l[kGlobal ? 1 : kSortMax];
    double *key = key_l;
    int *idx = idx_l;
    if (kGlobal) {
        const size_t P = (size_t)sort_len(a.n_max);
        key = reinterpret_cast<double *>(sort_ws) + (size_t)s * P * 2;
        idx = reinterpret_cast<int *>(key + P);
    }
    __shared__ double red_max[kT / 64], red_sum[kT / 64];
    int P = 1;
    while (P < N) P <<= 1;
    double lmax = 0.0, lsum = 0.0;
    for (int t = threadIdx.x; t < P; t += kT) {
        if (t < N) {
            const double r = R[j0 + t];
            key[t] = r;
            idx[t] = t;
            lmax = fmax(lmax, r);
            lsum += r;
        } else {
            key[t] = -1.0;
            idx[t] = 0x7fffffff;
        }
    }
    // block reductions (fixed order: deterministic)
    for (int o = 32; o > 0; o >>= 1) {
        lmax = fmax(lmax, __shfl_xor(lmax, o, 64));
        lsum += __shfl_xor(lsum, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red_max[threadIdx.x >> 6] = lmax;
        red_sum[threadIdx.x >> 6] = lsum;
    }
    __syncthreads();
    double rmax = 0.0, rsum = 0.0;
    for (int w = 0; w < kT / 64; ++w) {
        rmax = fmax(rmax, red_max[w]);
        rsum += red_sum[w];
    }
    const int limit = min(a.m0[s] + a.m_max, a.m_cap);
    const int per = (1 << dim) - 1;
    const bool failed = (a.stats && a.stats[s].status != PAM_ST_OK) || (a.flags[s] & 2);
    const bool stop = failed || !(rmax >= a.eps_tol) || a.round >= a.max_rounds || M >= limit;
    int nm = 0;
    if (!stop) {
        // bitonic sort, descending by key, ascending index on ties
        for (int k = 2; k <= P; k <<= 1) {
            for (int jj = k >> 1; jj > 0; jj >>= 1) {
                __syncthreads();
                for (int t = threadIdx.x; t < P; t += kT) {
                    const int ixj = t ^ jj;
                    if (ixj > t) {
                        const bool first_before = key[t] > key[ixj] || (key[t] == key[ixj] && idx[t] < idx[ixj]);
                        const bool desc = (t & k) == 0;
                        if (desc != first_before) {
                            const double tk = key[t]; key[t] = key[ixj]; key[ixj] = tk;
                            const int ti = idx[t]; idx[t] = idx[ixj]; idx[ixj] = ti;
                        }
                    }
                }
            }
        }
        __syncthreads();
        const int kt = min(a.k_top[s], N);
        // count eligible (R >= eps_tol) among the first kt ranks
        for (int r = 0; r < kt; ++r) {
            if (key[r] >= a.eps_tol) ++nm;
            else break;
        }
        const int n_add = min(nm, (limit - M) / per);
        const double sigma0 = a.sigma[(size_t)s * a.m_cap];
        for (int r = threadIdx.x; r < n_add; r += kT) {
            const int jl = idx[r];
            const int64_t jg = j0 + jl;
            const int l = a.elem_level[jg];
            double scale = 1.0, sw = sigma0;
            for (int i = 0; i <= l; ++i) {
                scale *= 0.5;
                sw *= a.eta;
            }
            for (int q = 1; q <= per; ++q) {
                const int mi = M + r * per + (q - 1);
                for (int d = 0; d < dim; ++d) {
                    const double o = (double)((q >> d) & 1);
                    const double off = (a.h[jg * dim + d] * scale) * o;  // exact: power of 2
                    a.c[((size_t)s * a.m_cap + mi) * dim + d] = a.x[jg * dim + d] + off;
                }
                a.sigma[(size_t)s * a.m_cap + mi] = sw;
                a.level[(size_t)s * a.m_cap + mi] = l + 1;
                a.beta[(size_t)s * a.m_cap + mi] = 0.0;
            }
            a.elem_level[jg] = l + 1;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            a.m[s] = M + n_add * per;
            if (n_add == 0) a.active[s] = 0;
        }
    } else if (threadIdx.x == 0) {
        a.active[s] = 0;
    }
    if (threadIdx.x == 0) {
        if (a.rounds) a.rounds[s] = a.round + 1;
        if (a.round_stats) {
            double *rs = a.round_stats + ((size_t)s * (a.max_rounds + 1) + a.round) * 7;
            rs[0] = M;
            rs[1] = a.stats ? a.stats[s].support : 0;
            rs[2] = rmax;
            rs[3] = nm;
            rs[4] = rsum;
            rs[5] = a.stats ? a.stats[s].stream_bytes : 0.0;
            rs[6] = a.stats ? a.stats[s].solve_us : 0.0;
        }
    }
}

pam_status mark_check_capacity(int n_max) {
    if (n_max > kSortMaxGlobal) {
        set_error("pam_refine: subdomains with more than 4194304 samples are not supported");
        return PAM_ERR_CAPACITY;
    }
    return PAM_OK;
}

size_t mark_ws_bytes(int n_sub, int n_max) {
    if (n_max <= kSortMax) return 0;
    return (size_t)n_sub * (size_t)sort_len(n_max) * (sizeof(double) + sizeof(int) + 4);
}

pam_status launch_mark_enrich(pam_ctx *ctx, const RefineArgs &a) {
    pam_status st = mark_check_capacity(a.n_max);
    if (st != PAM_OK) return st;
    if (a.n_max <= kSortMax) {
        hipLaunchKernelGGL(k_mark_enrich<false>, dim3(a.n_sub), dim3(kT), 0, ctx->stream, a,
                           wsp<double>(ctx, BUF_R), nullptr);
    } else {
        if ((st = ensure(ctx, BUF_MARK, mark_ws_bytes(a.n_sub, a.n_max))) != PAM_OK) return st;
        hipLaunchKernelGGL(k_mark_enrich<true>, dim3(a.n_sub), dim3(kT), 0, ctx->stream, a,
                           wsp<double>(ctx, BUF_R), wsp<char>(ctx, BUF_MARK));
    }
    PAM_CHECK_HIP(hipGetLastError());
    return PAM_OK;
}

}  // namespace pam
