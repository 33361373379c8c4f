// Global reconstruction kernels (gfx950): K*(x) = normalized expansion of
// the subdomain that owns x (Sec. 2 Step 4), at arbitrary query points.
//
// Queries are binned by owner (histogram, scan, scatter) so that a block
// evaluates up to kQ queries of one subdomain against that subdomain's
// centers, staged once in LDS and read as broadcasts. The per-query sums run
// in a fixed center order, so results do not depend on the binning order.
#include <float.h>

#include <string.h>

#include <algorithm>

#include "pam_internal.h"

namespace pam {

static constexpr int kE = 256;   // threads per block
static constexpr int kQ = 256;   // queries per chunk (one per thread)
static constexpr int kEC = 512;  // centers staged per pass

struct FieldDev {
    int32_t dim, n_sub_axis[3];
    int32_t axis_off;  // offset of the field's breakpoints in the axis table
    int32_t sub_base;
    int64_t q_begin, q_end;
};

struct EvalTables {
    const FieldDev *fields;
    const double *axis;
    int32_t n_fields;
};

template <typename TQ>
__device__ __forceinline__ int owner_of(const EvalTables &t, int f, const TQ *xq, int64_t q) {
    const FieldDev F = t.fields[f];
    int sub = 0, stride = 1, pos = F.axis_off;
    for (int d = 0; d < F.dim; ++d) {
        const double v = (double)xq[q * F.dim + d];
        const int n = F.n_sub_axis[d];
        const double *bx = t.axis + pos;
        if (!(v >= bx[0] && v <= bx[n])) return -1;
        int k = n - 1;  // last interval closed
        for (int i = 0; i < n; ++i)
            if (v < bx[i + 1]) { k = i; break; }
        sub += k * stride;
        stride *= n;
        pos += n + 1;
    }
    return F.sub_base + sub;
}

// Owner of every query and the per-subdomain query counts. Counts go to an
// LDS histogram per block and are flushed with one global atomic per
// touched bin (queries arrive in spatially coherent runs, so global atomics
// per query would serialize on a handful of counters).
static constexpr int kBinsLds = 8192;

template <typename TQ>
__global__ void __launch_bounds__(kE)
k_owner(EvalTables t, const TQ *__restrict__ xq, int64_t Q, int n_sub, int32_t *__restrict__ owner,
        int32_t *__restrict__ hist, TQ *__restrict__ out, unsigned long long *__restrict__ n_out) {
    __shared__ int32_t lh[kBinsLds];
    const bool local = n_sub <= kBinsLds;
    if (local)
        for (int b = threadIdx.x; b < n_sub; b += kE) lh[b] = 0;
    __syncthreads();
    for (int64_t q = (int64_t)blockIdx.x * kE + threadIdx.x; q < Q; q += (int64_t)gridDim.x * kE) {
        int f = 0;
        while (f + 1 < t.n_fields && q >= t.fields[f].q_end) ++f;
        int o = -1;
        if (q >= t.fields[f].q_begin && q < t.fields[f].q_end) o = owner_of(t, f, xq, q);
        owner[q] = o;
        if (o >= 0) {
            if (local) atomicAdd(&lh[o], 1);
            else atomicAdd(&hist[o], 1);
        } else {
            out[q] = (TQ)NAN;
            if (n_out) atomicAdd(n_out, 1ull);
        }
    }
    __syncthreads();
    if (local)
        for (int b = threadIdx.x; b < n_sub; b += kE)
            if (lh[b]) atomicAdd(&hist[b], lh[b]);
}

// Single-block exclusive scan of the owner histogram; also the chunk
// offsets (ceil(count / kQ) chunks per subdomain). cursor is cleared.
__global__ void __launch_bounds__(1024)
k_scan(int n_sub, const int32_t *__restrict__ hist, int64_t *__restrict__ base,
       int32_t *__restrict__ chunk_base, int32_t *__restrict__ cursor, int32_t *__restrict__ n_chunks) {
    __shared__ int64_t sh_q[1024];
    __shared__ int32_t sh_c[1024];
    __shared__ int64_t carry_q;
    __shared__ int32_t carry_c;
    if (threadIdx.x == 0) { carry_q = 0; carry_c = 0; }
    __syncthreads();
    for (int b0 = 0; b0 < n_sub; b0 += 1024) {
        const int i = b0 + threadIdx.x;
        const int32_t h = i < n_sub ? hist[i] : 0;
        sh_q[threadIdx.x] = h;
        sh_c[threadIdx.x] = (h + kQ - 1) / kQ;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            int64_t vq = 0;
            int32_t vc = 0;
            if ((int)threadIdx.x >= o) { vq = sh_q[threadIdx.x - o]; vc = sh_c[threadIdx.x - o]; }
            __syncthreads();
            sh_q[threadIdx.x] += vq;
            sh_c[threadIdx.x] += vc;
            __syncthreads();
        }
        if (i < n_sub) {
            base[i] = carry_q + sh_q[threadIdx.x] - h;
            chunk_base[i] = carry_c + sh_c[threadIdx.x] - (h + kQ - 1) / kQ;
            cursor[i] = 0;
        }
        __syncthreads();
        if (threadIdx.x == 1023) { carry_q += sh_q[1023]; carry_c += sh_c[1023]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) *n_chunks = carry_c;
}

// Binned positions: each block takes kScatter consecutive queries, ranks
// them inside their bins in LDS, reserves one range per touched bin with a
// global atomic, and writes the permutation.
static constexpr int kScatterPer = 16;
static constexpr int kScatter = kE * kScatterPer;

__global__ void __launch_bounds__(kE)
k_scatter(int64_t Q, int n_sub, const int32_t *__restrict__ owner, const int64_t *__restrict__ base,
          int32_t *__restrict__ cursor, int64_t *__restrict__ perm) {
    __shared__ int32_t lcount[kBinsLds];
    __shared__ int32_t lbase[kBinsLds];
    const int64_t q0 = (int64_t)blockIdx.x * kScatter;
    if (n_sub > kBinsLds) {
        for (int e = 0; e < kScatterPer; ++e) {
            const int64_t q = q0 + (int64_t)e * kE + threadIdx.x;
            if (q >= Q) break;
            const int o = owner[q];
            if (o < 0) continue;
            perm[base[o] + atomicAdd(&cursor[o], 1)] = q;
        }
        return;
    }
    for (int b = threadIdx.x; b < n_sub; b += kE) lcount[b] = 0;
    __syncthreads();
    int ow[kScatterPer], rk[kScatterPer];
#pragma unroll
    for (int e = 0; e < kScatterPer; ++e) {
        const int64_t q = q0 + (int64_t)e * kE + threadIdx.x;
        ow[e] = q < Q ? owner[q] : -1;
        rk[e] = ow[e] >= 0 ? atomicAdd(&lcount[ow[e]], 1) : 0;
    }
    __syncthreads();
    for (int b = threadIdx.x; b < n_sub; b += kE)
        if (lcount[b]) lbase[b] = atomicAdd(&cursor[b], lcount[b]);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kScatterPer; ++e) {
        const int64_t q = q0 + (int64_t)e * kE + threadIdx.x;
        if (ow[e] >= 0) perm[base[ow[e]] + lbase[ow[e]] + rk[e]] = q;
    }
}

// Chunk table: chunk c -> (subdomain, first binned position, count).
__global__ void __launch_bounds__(kE)
k_chunks(int n_sub, const int32_t *__restrict__ hist, const int64_t *__restrict__ base,
         const int32_t *__restrict__ chunk_base, int32_t *__restrict__ ch_sub,
         int64_t *__restrict__ ch_start, int32_t *__restrict__ ch_len) {
    const int s = blockIdx.x * kE + threadIdx.x;
    if (s >= n_sub) return;
    const int h = hist[s];
    const int nc = (h + kQ - 1) / kQ;
    for (int c = 0; c < nc; ++c) {
        const int id = chunk_base[s] + c;
        ch_sub[id] = s;
        ch_start[id] = base[s] + (int64_t)c * kQ;
        ch_len[id] = min(kQ, h - c * kQ);
    }
}

// Evaluation of one chunk. FP32 path: squared distance by direct differences
// in FP32 and phi = exp2(-r2 * log2(e) / (2 sigma^2)) with the hardware
// exp2; FP64 path: exp() of the FP64 exponent.
template <typename TQ>
__global__ void __launch_bounds__(kE)
k_eval_chunks(int dim, int m_cap, const int32_t *__restrict__ n_chunks,
              const int32_t *__restrict__ ch_sub, const int64_t *__restrict__ ch_start,
              const int32_t *__restrict__ ch_len, const int64_t *__restrict__ perm,
              const int32_t *__restrict__ m, const double *__restrict__ c,
              const double *__restrict__ sigma, const double *__restrict__ beta,
              const TQ *__restrict__ xq, TQ *__restrict__ out, int space) {
    const int ch = blockIdx.x;
    if (ch >= *n_chunks) return;
    const int s = ch_sub[ch];
    const int64_t start = ch_start[ch];
    const int len = ch_len[ch];
    const int M = max(0, min(m[s], m_cap));
    __shared__ TQ sc[kEC * 3];
    __shared__ TQ sa[kEC];
    __shared__ TQ sb[kEC];
    const bool live = (int)threadIdx.x < len;
    int64_t q = 0;
    TQ x[3] = {0, 0, 0};
    if (live) {
        q = perm[start + threadIdx.x];
        for (int d = 0; d < dim; ++d) x[d] = xq[q * dim + d];
    }
    TQ num = 0, den = 0;
    const double *cs = c + (size_t)s * m_cap * dim;
    for (int m0 = 0; m0 < M; m0 += kEC) {
        const int cnt = min(kEC, M - m0);
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += kE) {
            for (int d = 0; d < dim; ++d) sc[t * 3 + d] = (TQ)cs[(size_t)(m0 + t) * dim + d];
            const double sg = sigma[(size_t)s * m_cap + m0 + t];
            sa[t] = sizeof(TQ) == 4 ? (TQ)(1.4426950408889634 * 0.5 / (sg * sg)) : (TQ)(0.5 / (sg * sg));
            sb[t] = (TQ)beta[(size_t)s * m_cap + m0 + t];
        }
        __syncthreads();
        if (live) {
            if (dim == 2) {
#pragma unroll 4
                for (int t = 0; t < cnt; ++t) {
                    const TQ dx = x[0] - sc[t * 3], dy = x[1] - sc[t * 3 + 1];
                    const TQ r2 = dx * dx + dy * dy;
                    TQ p;
                    if constexpr (sizeof(TQ) == 4) p = __builtin_amdgcn_exp2f(-r2 * sa[t]);
                    else p = exp(-r2 * sa[t]);
                    num += sb[t] * p;
                    den += p;
                }
            } else {
                for (int t = 0; t < cnt; ++t) {
                    TQ r2 = 0;
                    for (int d = 0; d < dim; ++d) {
                        const TQ df = x[d] - sc[t * 3 + d];
                        r2 += df * df;
                    }
                    TQ p;
                    if constexpr (sizeof(TQ) == 4) p = __builtin_amdgcn_exp2f(-r2 * sa[t]);
                    else p = exp(-r2 * sa[t]);
                    num += sb[t] * p;
                    den += p;
                }
            }
        }
    }
    if (live) {
        TQ v = num / den;
        if (space == 1) {
            if constexpr (sizeof(TQ) == 4) v = exp10f(v);
            else v = exp10(v);
        }
        out[q] = v;
    }
}

// ---------------------------------------------------------------- launcher
pam_status launch_eval(pam_ctx *ctx, int n_fields, const pam_field *fields, const pam_dict *dict,
                       const double *beta, int dtype, const void *xq, int64_t Q, void *out,
                       int space, int64_t *n_outside) {
    // host tables
    int n_sub_total = 0;
    std::vector<FieldDev> fd(n_fields);
    std::vector<double> axis;
    for (int f = 0; f < n_fields; ++f) {
        const pam_field &F = fields[f];
        fd[f].dim = F.dim;
        int nsub = 1, pos = 0;
        for (int d = 0; d < 3; ++d) fd[f].n_sub_axis[d] = d < F.dim ? F.n_sub_axis[d] : 1;
        fd[f].axis_off = (int32_t)axis.size();
        for (int d = 0; d < F.dim; ++d) {
            for (int i = 0; i <= F.n_sub_axis[d]; ++i) axis.push_back(F.axis_x[pos + i]);
            pos += F.n_sub_axis[d] + 1;
            nsub *= F.n_sub_axis[d];
        }
        fd[f].sub_base = F.sub_base;
        fd[f].q_begin = F.q_begin;
        fd[f].q_end = F.q_end;
        n_sub_total = std::max(n_sub_total, F.sub_base + nsub);
    }
    const int64_t max_chunks = Q / kQ + n_sub_total + 1;
    // workspace layout inside BUF_EVAL
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o += (bytes + 255) / 256 * 256; return r; };
    const size_t o_fields = take(sizeof(FieldDev) * n_fields);
    const size_t o_axis = take(sizeof(double) * axis.size());
    const size_t o_owner = take(sizeof(int32_t) * Q);
    const size_t o_hist = take(sizeof(int32_t) * n_sub_total);
    const size_t o_base = take(sizeof(int64_t) * n_sub_total);
    const size_t o_cbase = take(sizeof(int32_t) * n_sub_total);
    const size_t o_cursor = take(sizeof(int32_t) * n_sub_total);
    const size_t o_nch = take(sizeof(int32_t));
    const size_t o_perm = take(sizeof(int64_t) * Q);
    const size_t o_chsub = take(sizeof(int32_t) * max_chunks);
    const size_t o_chstart = take(sizeof(int64_t) * max_chunks);
    const size_t o_chlen = take(sizeof(int32_t) * max_chunks);
    pam_status st = ensure(ctx, BUF_EVAL, o);
    if (st != PAM_OK) return st;
    char *w = wsp<char>(ctx, BUF_EVAL);
    // both tables in one staged upload
    std::vector<char> host(o_owner);
    memcpy(host.data() + o_fields, fd.data(), sizeof(FieldDev) * n_fields);
    memcpy(host.data() + o_axis, axis.data(), sizeof(double) * axis.size());
    if ((st = upload_to(ctx, w, host.data(), o_owner)) != PAM_OK) return st;
    PAM_CHECK_HIP(hipMemsetAsync(w + o_hist, 0, sizeof(int32_t) * n_sub_total, ctx->stream));
    EvalTables t;
    t.fields = (const FieldDev *)(w + o_fields);
    t.axis = (const double *)(w + o_axis);
    t.n_fields = n_fields;
    int32_t *owner = (int32_t *)(w + o_owner);
    int32_t *hist = (int32_t *)(w + o_hist);
    int64_t *base = (int64_t *)(w + o_base);
    int32_t *cbase = (int32_t *)(w + o_cbase);
    int32_t *cursor = (int32_t *)(w + o_cursor);
    int32_t *nch = (int32_t *)(w + o_nch);
    int64_t *perm = (int64_t *)(w + o_perm);
    int32_t *chsub = (int32_t *)(w + o_chsub);
    int64_t *chstart = (int64_t *)(w + o_chstart);
    int32_t *chlen = (int32_t *)(w + o_chlen);
    // owner pass: a few thousand resident blocks, each flushing one histogram
    const int grid_o = (int)std::max<int64_t>(1, std::min<int64_t>((Q + kE - 1) / kE, 2048));
    {
    KernelTimer kt_bin(ctx, PAM_TK_EVAL_BIN);
    if (Q > 0) {
        if (dtype == 0)
            hipLaunchKernelGGL((k_owner<float>), dim3(grid_o), dim3(kE), 0, ctx->stream, t,
                               (const float *)xq, Q, n_sub_total, owner, hist, (float *)out,
                               (unsigned long long *)n_outside);
        else
            hipLaunchKernelGGL((k_owner<double>), dim3(grid_o), dim3(kE), 0, ctx->stream, t,
                               (const double *)xq, Q, n_sub_total, owner, hist, (double *)out,
                               (unsigned long long *)n_outside);
        PAM_CHECK_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, ctx->stream, n_sub_total, hist, base, cbase,
                       cursor, nch);
    PAM_CHECK_HIP(hipGetLastError());
    if (Q > 0) {
        hipLaunchKernelGGL(k_scatter, dim3((unsigned)((Q + kScatter - 1) / kScatter)), dim3(kE), 0,
                           ctx->stream, Q, n_sub_total, owner, base, cursor, perm);
        PAM_CHECK_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_chunks, dim3((n_sub_total + kE - 1) / kE), dim3(kE), 0, ctx->stream,
                       n_sub_total, hist, base, cbase, chsub, chstart, chlen);
    PAM_CHECK_HIP(hipGetLastError());
    }
    KernelTimer kt_eval(ctx, PAM_TK_EVAL);
    if (Q > 0) {
        if (dtype == 0)
            hipLaunchKernelGGL((k_eval_chunks<float>), dim3((unsigned)max_chunks), dim3(kE), 0,
                               ctx->stream, dict->dim, dict->m_cap, nch, chsub, chstart, chlen,
                               perm, dict->m, dict->c, dict->sigma, beta, (const float *)xq,
                               (float *)out, space);
        else
            hipLaunchKernelGGL((k_eval_chunks<double>), dim3((unsigned)max_chunks), dim3(kE), 0,
                               ctx->stream, dict->dim, dict->m_cap, nch, chsub, chstart, chlen,
                               perm, dict->m, dict->c, dict->sigma, beta, (const double *)xq,
                               (double *)out, space);
        PAM_CHECK_HIP(hipGetLastError());
    }
    return PAM_OK;
}

}  // namespace pam
