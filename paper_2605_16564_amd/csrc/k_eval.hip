// Global reconstruction kernels (gfx950): K*(x) = normalized expansion of
// the subdomain that owns x (Sec. 2 Step 4), at arbitrary query points; the
// continuous variant that averages neighbouring local surrogates across
// interfaces (the remark after Step 4); and the interface jump of the
// piecewise field.
//
// Queries are binned by owner (histogram, scan, scatter) so that a block
// evaluates up to kQ queries of one subdomain against that subdomain's
// centers, staged once in LDS and read as broadcasts. The per-query sums run
// in a fixed center order, so results do not depend on the binning order.
//
// The continuous variant bins terms instead of queries: a query inside an
// interface band of width 2h has, per axis, its owner interval and one
// neighbour, so up to 2^dim (subdomain, weight) terms. Term c of query q
// (bit a of c set = neighbour on axis a) is evaluated like a query of that
// subdomain into slot q * 2^dim + c; a last pass sums the slots of each
// query in c order with the tensor-product weights.
#include <float.h>

#include <string.h>

#include <algorithm>

#include <mutex>

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
    int32_t n_axis;     // entries of the axis table
};

// The field and breakpoint tables in LDS when they fit: the owner search
// reads them once per axis and query, a chain of dependent loads.
static constexpr int kFieldsLds = 128;
static constexpr int kAxisLds = 4096;

__device__ __forceinline__ EvalTables stage_tables(const EvalTables &t, FieldDev *lf, double *la) {
    if (t.n_fields > kFieldsLds || t.n_axis > kAxisLds) return t;
    for (int i = threadIdx.x; i < t.n_fields; i += blockDim.x) lf[i] = t.fields[i];
    for (int i = threadIdx.x; i < t.n_axis; i += blockDim.x) la[i] = t.axis[i];
    __syncthreads();
    EvalTables l = t;
    l.fields = lf;
    l.axis = la;
    return l;
}

template <typename TQ, int DIM>
__device__ __forceinline__ int owner_of(const EvalTables &t, int f, const TQ *xq, int64_t q) {
    const FieldDev F = t.fields[f];
    int sub = 0, stride = 1, pos = F.axis_off;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const double v = (double)xq[q * DIM + d];
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

// Interface weights. At interior breakpoint b_i the band half-width is
// h_i = blend * min(L_{i-1}, L_i) (L = interval lengths); in the band the
// interval on the left has weight 1 - rho(s) and the one on the right rho(s),
// s = (t - b_i + h_i) / (2 h_i), with the C1 ramp rho(s) = s^2 (3 - 2 s).
// blend <= 1/2 keeps the two bands of an interval apart, so a point sees its
// owner interval and at most one neighbour per axis.
struct AxisTerm {
    int k;          // owner interval
    int nb;         // neighbour offset: -1, +1, or 0 (none)
    double w_own, w_nb;
};

// The band tests and weights are evaluated with contraction off, so that the
// term, scatter and combine passes take identical decisions and weights.
__device__ __forceinline__ double ramp(double s) {
#pragma clang fp contract(off)
    return s <= 0.0 ? 0.0 : (s >= 1.0 ? 1.0 : s * s * (3.0 - 2.0 * s));
}

// Per-axis terms of query q of field f; returns the owner subdomain (field
// local) or -1 outside the closed domain.
// DIM is the fields' dimension (one per launch), so that the per-axis state
// stays in registers.
template <typename TQ, int DIM>
__device__ __forceinline__ int axis_terms(const EvalTables &t, int f, const TQ *xq, int64_t q,
                                          double blend, AxisTerm *at, int *stride_out) {
#pragma clang fp contract(off)
    const FieldDev F = t.fields[f];
    int sub = 0, stride = 1, pos = F.axis_off;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const double v = (double)xq[q * DIM + d];
        const int n = F.n_sub_axis[d];
        const double *bx = t.axis + pos;
        if (!(v >= bx[0] && v <= bx[n])) return -1;
        int k = n - 1;
        for (int i = 0; i < n; ++i)
            if (v < bx[i + 1]) { k = i; break; }
        AxisTerm a{k, 0, 1.0, 0.0};
        if (k + 1 < n) {   // band at the right breakpoint
            const double h = blend * fmin(bx[k + 1] - bx[k], bx[k + 2] - bx[k + 1]);
            if (h > 0.0 && v > bx[k + 1] - h) {
                const double r = ramp((v - (bx[k + 1] - h)) / (2.0 * h));
                a.nb = 1;
                a.w_own = 1.0 - r;
                a.w_nb = r;
            }
        }
        if (k > 0 && a.nb == 0) {   // band at the left breakpoint
            const double h = blend * fmin(bx[k] - bx[k - 1], bx[k + 1] - bx[k]);
            if (h > 0.0 && v < bx[k] + h) {
                const double r = ramp((v - (bx[k] - h)) / (2.0 * h));
                a.nb = -1;
                a.w_own = r;
                a.w_nb = 1.0 - r;
            }
        }
        at[d] = a;
        stride_out[d] = stride;
        sub += k * stride;
        stride *= n;
        pos += n + 1;
    }
    return sub;
}

// Term c of a query with axis terms at: weight and subdomain offset from the
// owner, or -1 if the term is absent. A term exists when the query lies
// strictly inside the band of every axis its bits select (a decision taken
// by comparisons only, so every pass agrees on it); its weight may still
// round to 0 at a band edge and then adds nothing.
template <int DIM>
__device__ __forceinline__ double term_weight(const AxisTerm *at, const int *stride, int c,
                                              int *dsub) {
#pragma clang fp contract(off)
    double w = 1.0;
    int o = 0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        if ((c >> d) & 1) {
            if (at[d].nb == 0) return -1.0;
            w *= at[d].w_nb;
            o += at[d].nb * stride[d];
        } else {
            w *= at[d].w_own;
        }
    }
    *dsub = o;
    return w;
}

// Field of query q: the first f with q < q_end(f) (ranges tile [0, Q) in
// order), by binary search, clamped to the last field.
__device__ __forceinline__ int field_of(const EvalTables &t, int64_t q) {
    int lo = 0, hi = t.n_fields - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (q < t.fields[mid].q_end) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// Owner of every query and the per-subdomain query counts. Counts go to an
// LDS histogram per block and are flushed with one global atomic per
// touched bin (queries arrive in spatially coherent runs, so global atomics
// per query would serialize on a handful of counters).
static constexpr int kBinsLds = 8192;

template <typename TQ, int DIM>
__global__ void __launch_bounds__(kE)
k_owner(EvalTables tg, const TQ *__restrict__ xq, int64_t Q, int n_sub, int32_t *__restrict__ owner,
        int32_t *__restrict__ hist, TQ *__restrict__ out, unsigned long long *__restrict__ n_out) {
    __shared__ int32_t lh[kBinsLds];
    __shared__ FieldDev lf[kFieldsLds];
    __shared__ double la[kAxisLds];
    const EvalTables t = stage_tables(tg, lf, la);
    const bool local = n_sub <= kBinsLds;
    if (local)
        for (int b = threadIdx.x; b < n_sub; b += kE) lh[b] = 0;
    __syncthreads();
    for (int64_t q = (int64_t)blockIdx.x * kE + threadIdx.x; q < Q; q += (int64_t)gridDim.x * kE) {
        const int f = field_of(t, q);
        int o = -1;
        if (q >= t.fields[f].q_begin && q < t.fields[f].q_end) o = owner_of<TQ, DIM>(t, f, xq, q);
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

// Binned positions: each block takes `per` consecutive queries per thread
// in two sweeps over owner[]: the first counts them per bin in LDS and
// reserves one range per touched bin with a global atomic, the second ranks
// them inside the block's range and writes the permutation. `per` grows with
// the number of bins so that clearing and flushing the LDS bins stays a small
// part of a block's work.
__global__ void __launch_bounds__(kE)
k_scatter(int64_t Q, int n_sub, int per, const int32_t *__restrict__ owner,
          const int64_t *__restrict__ base, int32_t *__restrict__ cursor,
          int64_t *__restrict__ perm) {
    __shared__ int32_t lcount[kBinsLds];
    __shared__ int32_t lbase[kBinsLds];
    const int64_t q0 = (int64_t)blockIdx.x * kE * per;
    const int64_t q1 = min(Q, q0 + (int64_t)kE * per);
    if (n_sub > kBinsLds) {
        for (int64_t q = q0 + threadIdx.x; q < q1; q += kE) {
            const int o = owner[q];
            if (o >= 0) perm[base[o] + atomicAdd(&cursor[o], 1)] = q;
        }
        return;
    }
    for (int b = threadIdx.x; b < n_sub; b += kE) lcount[b] = 0;
    __syncthreads();
    for (int64_t q = q0 + threadIdx.x; q < q1; q += kE) {
        const int o = owner[q];
        if (o >= 0) atomicAdd(&lcount[o], 1);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < n_sub; b += kE) {
        const int n = lcount[b];
        lbase[b] = n ? atomicAdd(&cursor[b], n) : 0;
        lcount[b] = 0;
    }
    __syncthreads();
    for (int64_t q = q0 + threadIdx.x; q < q1; q += kE) {
        const int o = owner[q];
        if (o >= 0) perm[base[o] + lbase[o] + atomicAdd(&lcount[o], 1)] = q;
    }
}

// Continuous variant, pass 1: terms of every query and the per-subdomain
// term counts (LDS histogram as in k_owner). Outside points get NaN.
template <typename TQ, int DIM>
__global__ void __launch_bounds__(kE)
k_terms(EvalTables tg, const TQ *__restrict__ xq, int64_t Q, int n_sub, double blend,
        int32_t *__restrict__ hist, TQ *__restrict__ out, unsigned long long *__restrict__ n_out) {
    __shared__ int32_t lh[kBinsLds];
    __shared__ FieldDev lf[kFieldsLds];
    __shared__ double la[kAxisLds];
    const EvalTables t = stage_tables(tg, lf, la);
    const bool local = n_sub <= kBinsLds;
    if (local)
        for (int b = threadIdx.x; b < n_sub; b += kE) lh[b] = 0;
    __syncthreads();
    for (int64_t q = (int64_t)blockIdx.x * kE + threadIdx.x; q < Q; q += (int64_t)gridDim.x * kE) {
        const int f = field_of(t, q);
        AxisTerm at[DIM];
        int stride[DIM];
        int o = -1;
        if (q >= t.fields[f].q_begin && q < t.fields[f].q_end)
            o = axis_terms<TQ, DIM>(t, f, xq, q, blend, at, stride);
        if (o < 0) {
            out[q] = (TQ)NAN;
            if (n_out) atomicAdd(n_out, 1ull);
            continue;
        }
        o += t.fields[f].sub_base;
#pragma unroll
        for (int c = 0; c < (1 << DIM); ++c) {
            int ds = 0;
            if (term_weight<DIM>(at, stride, c, &ds) >= 0.0) {
                if (local) atomicAdd(&lh[o + ds], 1);
                else atomicAdd(&hist[o + ds], 1);
            }
        }
    }
    __syncthreads();
    if (local)
        for (int b = threadIdx.x; b < n_sub; b += kE)
            if (lh[b]) atomicAdd(&hist[b], lh[b]);
}

// Continuous variant, pass 2: binned positions of the terms (term id
// q * 2^dim + c). A block takes kTermBlk consecutive queries in two sweeps
// that recompute the terms bit-identically to pass 1: the first counts them
// per bin in LDS and reserves one range per touched bin with a global
// atomic, the second ranks them inside the block's range and writes the
// permutation (the order inside a bin does not matter: every term has its
// own slot).
static constexpr int kTermPer = 8;                 // queries per thread
static constexpr int kTermBlk = kE * kTermPer;     // queries per block

template <typename TQ, int DIM>
__device__ __forceinline__ int query_terms(const EvalTables &t, const TQ *xq, int64_t Q, double blend,
                                           int64_t q, int *sub) {
    if (q >= Q) return 0;
    const int f = field_of(t, q);
    if (q < t.fields[f].q_begin || q >= t.fields[f].q_end) return 0;
    AxisTerm at[DIM];
    int stride[DIM];
    const int o = axis_terms<TQ, DIM>(t, f, xq, q, blend, at, stride);
    if (o < 0) return 0;
    int mask = 0;
#pragma unroll
    for (int c = 0; c < (1 << DIM); ++c) {
        int ds = 0;
        sub[c] = 0;
        if (term_weight<DIM>(at, stride, c, &ds) >= 0.0) {
            sub[c] = t.fields[f].sub_base + o + ds;
            mask |= 1 << c;
        }
    }
    return mask;
}

template <typename TQ, int DIM>
__global__ void __launch_bounds__(kE)
k_scatter_terms(EvalTables t, const TQ *__restrict__ xq, int64_t Q, int n_sub, double blend,
                const int64_t *__restrict__ base, int32_t *__restrict__ cursor,
                int64_t *__restrict__ perm) {
    __shared__ int32_t lcount[kBinsLds];
    __shared__ int32_t lbase[kBinsLds];
    const bool local = n_sub <= kBinsLds;
    const int64_t q0 = (int64_t)blockIdx.x * kTermBlk;
    if (!local) {
        for (int e = 0; e < kTermPer; ++e) {
            const int64_t q = q0 + (int64_t)e * kE + threadIdx.x;
            int sub[1 << DIM];
            const int mask = query_terms<TQ, DIM>(t, xq, Q, blend, q, sub);
#pragma unroll
            for (int c = 0; c < (1 << DIM); ++c)
                if ((mask >> c) & 1)
                    perm[base[sub[c]] + atomicAdd(&cursor[sub[c]], 1)] = (q << DIM) | c;
        }
        return;
    }
    for (int b = threadIdx.x; b < n_sub; b += kE) lcount[b] = 0;
    __syncthreads();
    for (int e = 0; e < kTermPer; ++e) {
        const int64_t q = q0 + (int64_t)e * kE + threadIdx.x;
        int sub[1 << DIM];
        const int mask = query_terms<TQ, DIM>(t, xq, Q, blend, q, sub);
#pragma unroll
        for (int c = 0; c < (1 << DIM); ++c)
            if ((mask >> c) & 1) atomicAdd(&lcount[sub[c]], 1);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < n_sub; b += kE) {
        const int n = lcount[b];
        lbase[b] = n ? atomicAdd(&cursor[b], n) : 0;
        lcount[b] = 0;
    }
    __syncthreads();
    for (int e = 0; e < kTermPer; ++e) {
        const int64_t q = q0 + (int64_t)e * kE + threadIdx.x;
        int sub[1 << DIM];
        const int mask = query_terms<TQ, DIM>(t, xq, Q, blend, q, sub);
#pragma unroll
        for (int c = 0; c < (1 << DIM); ++c)
            if ((mask >> c) & 1) {
                const int r = atomicAdd(&lcount[sub[c]], 1);
                perm[base[sub[c]] + lbase[sub[c]] + r] = (q << DIM) | c;
            }
    }
}

// Continuous variant, pass 4: out[q] = sum_c w_c K*_{sub(c)}(x_q) over the
// present terms in c order (FP64 weights and sum), then 10^ if asked.
template <typename TQ, int DIM>
__global__ void __launch_bounds__(kE)
k_combine(EvalTables tg, const TQ *__restrict__ xq, int64_t Q, double blend,
          const TQ *__restrict__ tval, TQ *__restrict__ out, int space) {
    __shared__ FieldDev lf[kFieldsLds];
    __shared__ double la[kAxisLds];
    const EvalTables t = stage_tables(tg, lf, la);
    for (int64_t q = (int64_t)blockIdx.x * kE + threadIdx.x; q < Q; q += (int64_t)gridDim.x * kE) {
        const int f = field_of(t, q);
        if (q < t.fields[f].q_begin || q >= t.fields[f].q_end) continue;
        AxisTerm at[DIM];
        int stride[DIM];
        if (axis_terms<TQ, DIM>(t, f, xq, q, blend, at, stride) < 0) continue;
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < (1 << DIM); ++c) {
            int ds = 0;
            const double w = term_weight<DIM>(at, stride, c, &ds);
            if (w >= 0.0) acc += w * (double)tval[(q << DIM) | c];
        }
        TQ v = (TQ)acc;
        if (space == 1) {
            if constexpr (sizeof(TQ) == 4) v = exp10f(v);
            else v = exp10(v);
        }
        out[q] = v;
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
// TERMS: perm holds term ids (q * 2^dim + c); the normalized value goes to
// slot tval[id] with no output transform.
template <typename TQ, bool TERMS>
__global__ void __launch_bounds__(kE)
k_eval_chunks(int dim, int m_cap, const int32_t *__restrict__ n_chunks,
              const int32_t *__restrict__ ch_sub, const int64_t *__restrict__ ch_start,
              const int32_t *__restrict__ ch_len, const int64_t *__restrict__ perm,
              const int32_t *__restrict__ m, const double *__restrict__ c,
              const double *__restrict__ sigma, const double *__restrict__ beta,
              const TQ *__restrict__ xq, TQ *__restrict__ out, int space,
              TQ *__restrict__ tval, int plain) {
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
    int64_t q = 0, id = 0;
    TQ x[3] = {0, 0, 0};
    if (live) {
        id = perm[start + threadIdx.x];
        q = TERMS ? id >> dim : id;
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
        TQ v = plain ? num : num / den;
        if constexpr (TERMS) {
            tval[id] = v;
        } else {
            if (space == 1) {
                if constexpr (sizeof(TQ) == 4) v = exp10f(v);
                else v = exp10(v);
            }
            out[q] = v;
        }
    }
}

// ---------------------------------------------------------------- launcher
namespace {

// Host tables of the fields: per-field descriptors and the concatenated
// breakpoint coordinates; returns the number of subdomains they span.
int field_tables(int n_fields, const pam_field *fields, std::vector<FieldDev> &fd,
                 std::vector<double> &axis) {
    int n_sub_total = 0;
    fd.resize(n_fields);
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
    return n_sub_total;
}

// The no-alloc evaluation passes its small tables by value (one kernel
// argument) and clears the histogram in the same kernel.
static constexpr int kNaFields = 8, kNaAxis = 240;
struct TablesArg {
    FieldDev f[kNaFields];
    double axis[kNaAxis];
    int32_t n_fields, n_axis, n_sub;
};

__global__ void __launch_bounds__(kE)
k_put_tables(TablesArg t, FieldDev *__restrict__ fd, double *__restrict__ ax, int32_t *__restrict__ hist) {
    const int i = blockIdx.x * kE + threadIdx.x;
    const int stride = gridDim.x * kE;
    for (int k = i; k < t.n_fields; k += stride) fd[k] = t.f[k];
    for (int k = i; k < t.n_axis; k += stride) ax[k] = t.axis[k];
    for (int k = i; k < t.n_sub; k += stride) hist[k] = 0;
}

// The same tables in the fixed arrays of TablesArg (no host containers);
// returns the number of subdomains, or -1 beyond kNaFields / kNaAxis.
int field_tables_fixed(int n_fields, const pam_field *fields, TablesArg &t) {
    memset(&t, 0, sizeof(t));
    if (n_fields > kNaFields) return -1;
    int n_sub_total = 0, na = 0;
    for (int f = 0; f < n_fields; ++f) {
        const pam_field &F = fields[f];
        FieldDev &d = t.f[f];
        d.dim = F.dim;
        int nsub = 1, pos = 0;
        for (int a = 0; a < 3; ++a) d.n_sub_axis[a] = a < F.dim ? F.n_sub_axis[a] : 1;
        d.axis_off = na;
        for (int a = 0; a < F.dim; ++a) {
            if (na + F.n_sub_axis[a] + 1 > kNaAxis) return -1;
            for (int i = 0; i <= F.n_sub_axis[a]; ++i) t.axis[na++] = F.axis_x[pos + i];
            pos += F.n_sub_axis[a] + 1;
            nsub *= F.n_sub_axis[a];
        }
        d.sub_base = F.sub_base;
        d.q_begin = F.q_begin;
        d.q_end = F.q_end;
        n_sub_total = std::max(n_sub_total, F.sub_base + nsub);
    }
    t.n_fields = n_fields;
    t.n_axis = na;
    t.n_sub = n_sub_total;
    return n_sub_total;
}

template <typename TQ>
pam_status eval_typed(pam_ctx *ctx, int n_fields, const pam_field *fields, const pam_dict *dict,
                      const double *beta, bool blended, double blend, const TQ *xq, int64_t Q,
                      TQ *out, int space, int64_t *n_outside, char *ext_ws = nullptr,
                      size_t ext_cap = 0) {
    std::vector<FieldDev> fd;
    std::vector<double> axis;
    TablesArg ta;   // the no-alloc path's tables (no host containers either)
    int n_sub_total = 0;
    size_t n_axis = 0;
    if (ext_ws) {
        n_sub_total = field_tables_fixed(n_fields, fields, ta);
        if (n_sub_total < 0) {
            set_error("pam_eval_noalloc: more than 8 fields or 240 breakpoints");
            return PAM_ERR_CAPACITY;
        }
        n_axis = (size_t)ta.n_axis;
    } else {
        n_sub_total = field_tables(n_fields, fields, fd, axis);
        n_axis = axis.size();
    }
    int dim_max = 1;
    for (int f = 0; f < n_fields; ++f) dim_max = std::max(dim_max, fields[f].dim);
    // binned items: queries, or term slots (2^dim per query) in the continuous variant
    const int64_t slots = blended ? Q << dim_max : Q;
    const int64_t max_chunks = slots / kQ + n_sub_total + 1;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o += (bytes + 255) / 256 * 256; return r; };
    const size_t o_fields = take(sizeof(FieldDev) * n_fields);
    const size_t o_axis = take(sizeof(double) * n_axis);
    const size_t o_owner = take(blended ? 0 : sizeof(int32_t) * Q);
    const size_t o_hist = take(sizeof(int32_t) * n_sub_total);
    const size_t o_base = take(sizeof(int64_t) * n_sub_total);
    const size_t o_cbase = take(sizeof(int32_t) * n_sub_total);
    const size_t o_cursor = take(sizeof(int32_t) * n_sub_total);
    const size_t o_nch = take(sizeof(int32_t));
    const size_t o_perm = take(sizeof(int64_t) * slots);
    const size_t o_chsub = take(sizeof(int32_t) * max_chunks);
    const size_t o_chstart = take(sizeof(int64_t) * max_chunks);
    const size_t o_chlen = take(sizeof(int32_t) * max_chunks);
    const size_t o_tval = take(blended ? sizeof(TQ) * slots : 0);
    pam_status st;
    char *w;
    const bool timed = ext_ws == nullptr;   // the no-alloc path creates no timing events
    if (ext_ws) {
        if (o > ext_cap) {
            set_error("pam_eval_noalloc: the binning workspace of this call exceeds the fixed 64 MiB "
                      "(about 12 B per query plus 24 B per subdomain)");
            return PAM_ERR_CAPACITY;
        }
        w = ext_ws;
        const int nb = (int)std::min<int64_t>(64, (std::max<int64_t>(n_sub_total, kNaAxis) + kE - 1) / kE);
        hipLaunchKernelGGL(k_put_tables, dim3(nb), dim3(kE), 0, ctx->stream, ta, (FieldDev *)(w + o_fields),
                           (double *)(w + o_axis), (int32_t *)(w + o_hist));
        PAM_CHECK_HIP(hipGetLastError());
    } else {
        if ((st = ensure(ctx, BUF_EVAL, o)) != PAM_OK) return st;
        w = wsp<char>(ctx, BUF_EVAL);
        // both tables in one staged upload
        std::vector<char> host(o_owner);
        memcpy(host.data() + o_fields, fd.data(), sizeof(FieldDev) * n_fields);
        memcpy(host.data() + o_axis, axis.data(), sizeof(double) * axis.size());
        if ((st = upload_to(ctx, w, host.data(), o_owner)) != PAM_OK) return st;
        PAM_CHECK_HIP(hipMemsetAsync(w + o_hist, 0, sizeof(int32_t) * n_sub_total, ctx->stream));
    }
    EvalTables t;
    t.fields = (const FieldDev *)(w + o_fields);
    t.axis = (const double *)(w + o_axis);
    t.n_fields = n_fields;
    t.n_axis = (int32_t)n_axis;
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
    TQ *tval = (TQ *)(w + o_tval);
    auto *n_out = (unsigned long long *)n_outside;
    // owner / term pass: a few thousand resident blocks, each flushing one histogram
    // owner / term histograms: every block flushes one global atomic per
    // touched bin, so the grid is kept at 2 blocks per CU to bound the
    // contention on the few bins that spatially coherent queries touch
    const int grid_o = (int)std::max<int64_t>(1, std::min<int64_t>((Q + kE - 1) / kE, 512));
    {
        KernelTimer kt_bin(ctx, timed ? PAM_TK_EVAL_BIN : -1);
        if (Q > 0) {
            if (blended) {
                auto kt = dim_max == 1 ? k_terms<TQ, 1> : dim_max == 2 ? k_terms<TQ, 2> : k_terms<TQ, 3>;
                hipLaunchKernelGGL(kt, dim3(grid_o), dim3(kE), 0, ctx->stream, t, xq, Q, n_sub_total,
                                   blend, hist, out, n_out);
            } else {
                auto ko = dim_max == 1 ? k_owner<TQ, 1> : dim_max == 2 ? k_owner<TQ, 2> : k_owner<TQ, 3>;
                hipLaunchKernelGGL(ko, dim3(grid_o), dim3(kE), 0, ctx->stream, t, xq, Q, n_sub_total,
                                   owner, hist, out, n_out);
            }
            PAM_CHECK_HIP(hipGetLastError());
        }
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, ctx->stream, n_sub_total, hist, base,
                           cbase, cursor, nch);
        PAM_CHECK_HIP(hipGetLastError());
        if (Q > 0) {
            if (blended) {
                auto ks = dim_max == 1 ? k_scatter_terms<TQ, 1>
                        : dim_max == 2 ? k_scatter_terms<TQ, 2> : k_scatter_terms<TQ, 3>;
                hipLaunchKernelGGL(ks, dim3((unsigned)((Q + kTermBlk - 1) / kTermBlk)), dim3(kE), 0,
                                   ctx->stream, t, xq, Q, n_sub_total, blend, base, cursor, perm);
            } else {
                const int per = std::min(256, std::max(16, (4 * n_sub_total + kE - 1) / kE));
                const int64_t span = (int64_t)kE * per;
                hipLaunchKernelGGL(k_scatter, dim3((unsigned)((Q + span - 1) / span)), dim3(kE), 0,
                                   ctx->stream, Q, n_sub_total, per, owner, base, cursor, perm);
            }
            PAM_CHECK_HIP(hipGetLastError());
        }
        hipLaunchKernelGGL(k_chunks, dim3((n_sub_total + kE - 1) / kE), dim3(kE), 0, ctx->stream,
                           n_sub_total, hist, base, cbase, chsub, chstart, chlen);
        PAM_CHECK_HIP(hipGetLastError());
    }
    if (Q == 0) return PAM_OK;
    {
        KernelTimer kt_eval(ctx, !timed ? -1 : blended ? PAM_TK_BLEND : PAM_TK_EVAL);
        if (blended)
            hipLaunchKernelGGL((k_eval_chunks<TQ, true>), dim3((unsigned)max_chunks), dim3(kE), 0,
                               ctx->stream, dict->dim, dict->m_cap, nch, chsub, chstart, chlen,
                               perm, dict->m, dict->c, dict->sigma, beta, xq, out, space, tval,
                               dict->basis == PAM_BASIS_PLAIN);
        else
            hipLaunchKernelGGL((k_eval_chunks<TQ, false>), dim3((unsigned)max_chunks), dim3(kE), 0,
                               ctx->stream, dict->dim, dict->m_cap, nch, chsub, chstart, chlen,
                               perm, dict->m, dict->c, dict->sigma, beta, xq, out, space, tval,
                               dict->basis == PAM_BASIS_PLAIN);
        PAM_CHECK_HIP(hipGetLastError());
    }
    if (blended) {
        // the weighted sum is bookkeeping like the binning: timed with it
        KernelTimer kt_comb(ctx, timed ? PAM_TK_EVAL_BIN : -1);
        auto kc = dim_max == 1 ? k_combine<TQ, 1> : dim_max == 2 ? k_combine<TQ, 2> : k_combine<TQ, 3>;
        hipLaunchKernelGGL(kc, dim3(grid_o), dim3(kE), 0, ctx->stream, t, xq, Q, blend,
                           (const TQ *)tval, out, space);
        PAM_CHECK_HIP(hipGetLastError());
    }
    return PAM_OK;
}

}  // namespace

pam_status launch_eval(pam_ctx *ctx, int n_fields, const pam_field *fields, const pam_dict *dict,
                       const double *beta, int dtype, const void *xq, int64_t Q, void *out,
                       int space, int64_t *n_outside) {
    if (dtype == 0)
        return eval_typed(ctx, n_fields, fields, dict, beta, false, 0.0, (const float *)xq, Q,
                          (float *)out, space, n_outside);
    return eval_typed(ctx, n_fields, fields, dict, beta, false, 0.0, (const double *)xq, Q,
                      (double *)out, space, n_outside);
}

// ---------------------------------------------------------------- no-alloc evaluation
// The binning workspace of pam_eval_noalloc: one fixed array per GPU, held
// until the process ends. Host code never uses this name as an address: the
// device address of each GPU's copy comes from hipGetSymbolAddress, taken
// once per device with that device current (eval_scratch_init, called from
// pam_create) and kept in g_scratch.
static constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch[kMaxDevices] = {};

pam_status eval_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) {
        set_error("device index beyond the scratch table");
        return PAM_ERR_ARG;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[device]) return PAM_OK;
    int cur = -1;
    PAM_CHECK_HIP(hipGetDevice(&cur));
    if (cur != device) {
        set_error("eval_scratch_init: the device is not current");
        return PAM_ERR_STATE;
    }
    void *ptr = nullptr;
    PAM_CHECK_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch[device] = ptr;
    return PAM_OK;
}

pam_status launch_eval_noalloc(pam_ctx *ctx, int n_fields, const pam_field *fields,
                               const pam_dict *dict, const double *beta, int dtype, const void *xq,
                               int64_t Q, void *out, int space, int64_t *n_outside) {
    void *ws = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        ws = ctx->device >= 0 && ctx->device < kMaxDevices ? g_scratch[ctx->device] : nullptr;
    }
    if (!ws) {
        set_error("pam_eval_noalloc: the scratch array of this device was not set up");
        return PAM_ERR_STATE;
    }
    if (dtype == 0)
        return eval_typed(ctx, n_fields, fields, dict, beta, false, 0.0, (const float *)xq, Q,
                          (float *)out, space, n_outside, (char *)ws, kScratchBytes);
    return eval_typed(ctx, n_fields, fields, dict, beta, false, 0.0, (const double *)xq, Q,
                      (double *)out, space, n_outside, (char *)ws, kScratchBytes);
}

pam_status launch_eval_blend(pam_ctx *ctx, int n_fields, const pam_field *fields,
                             const pam_dict *dict, const double *beta, double blend, int dtype,
                             const void *xq, int64_t Q, void *out, int space, int64_t *n_outside) {
    if (dtype == 0)
        return eval_typed(ctx, n_fields, fields, dict, beta, true, blend, (const float *)xq, Q,
                          (float *)out, space, n_outside);
    return eval_typed(ctx, n_fields, fields, dict, beta, true, blend, (const double *)xq, Q,
                      (double *)out, space, n_outside);
}

// ---------------------------------------------------------------- interface jump
// One block per interior interface piece: the face shared by subdomains A
// and B = A + e_axis, sampled at the midpoints of an n-per-axis subdivision;
// both local surrogates in FP64 (centers of A, then of B, staged in LDS).
struct FaceDev {
    int32_t a_sub, b_sub, axis, dim;
    double lo[3], hi[3];   // B's owned box; the face lies at lo[axis]
};

static constexpr int kJT = 256;

__global__ void __launch_bounds__(kJT)
k_jump(const FaceDev *__restrict__ faces, int n_faces, int n, int m_cap,
       const int32_t *__restrict__ m, const double *__restrict__ c,
       const double *__restrict__ sigma, const double *__restrict__ beta,
       double *__restrict__ out, int plain) {
    const int f = blockIdx.x;
    if (f >= n_faces) return;
    const FaceDev F = faces[f];
    const int dim = F.dim;
    int n_pts = 1;
    for (int b = 0; b < dim - 1; ++b) n_pts *= n;
    __shared__ double sc[kEC * 3];
    __shared__ double sa[kEC];
    __shared__ double sb[kEC];
    __shared__ double red_max[kJT], red_sum[kJT];
    double mx = 0.0, sum = 0.0;
    for (int p0 = 0; p0 < n_pts; p0 += kJT) {
        const int p = p0 + threadIdx.x;
        const bool live = p < n_pts;
        double x[3] = {0.0, 0.0, 0.0};
        int rest = p;
        for (int b = 0; b < dim; ++b) {
            if (b == F.axis) {
                x[b] = F.lo[b];
            } else {
                const int j = rest % n;
                rest /= n;
                x[b] = F.lo[b] + (j + 0.5) * (F.hi[b] - F.lo[b]) / n;
            }
        }
        double val[2];
        for (int side = 0; side < 2; ++side) {
            const int s = side == 0 ? F.a_sub : F.b_sub;
            const int M = max(0, min(m[s], m_cap));
            double num = 0.0, den = 0.0;
            for (int m0 = 0; m0 < M; m0 += kEC) {
                const int cnt = min(kEC, M - m0);
                __syncthreads();
                for (int t = threadIdx.x; t < cnt; t += kJT) {
                    for (int d = 0; d < dim; ++d)
                        sc[t * 3 + d] = c[((size_t)s * m_cap + m0 + t) * dim + d];
                    const double sg = sigma[(size_t)s * m_cap + m0 + t];
                    sa[t] = 0.5 / (sg * sg);
                    sb[t] = beta[(size_t)s * m_cap + m0 + t];
                }
                __syncthreads();
                if (live) {
                    for (int t = 0; t < cnt; ++t) {
                        double r2 = 0.0;
                        for (int d = 0; d < dim; ++d) {
                            const double df = x[d] - sc[t * 3 + d];
                            r2 += df * df;
                        }
                        const double ph = exp(-r2 * sa[t]);
                        num += sb[t] * ph;
                        den += ph;
                    }
                }
            }
            val[side] = plain ? num : num / den;
        }
        if (live) {
            const double j = fabs(val[0] - val[1]);
            mx = fmax(mx, j);
            sum += j;
        }
    }
    red_max[threadIdx.x] = mx;
    red_sum[threadIdx.x] = sum;
    __syncthreads();
    for (int k = kJT / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            red_max[threadIdx.x] = fmax(red_max[threadIdx.x], red_max[threadIdx.x + k]);
            red_sum[threadIdx.x] += red_sum[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * (size_t)f] = red_max[0];
        out[2 * (size_t)f + 1] = red_sum[0] / n_pts;
    }
}

int64_t interface_count(int n_fields, const pam_field *fields) {
    int64_t n = 0;
    for (int f = 0; f < n_fields; ++f) {
        int64_t tot = 1;
        for (int d = 0; d < fields[f].dim; ++d) tot *= fields[f].n_sub_axis[d];
        for (int d = 0; d < fields[f].dim; ++d)
            n += tot / fields[f].n_sub_axis[d] * (fields[f].n_sub_axis[d] - 1);
    }
    return n;
}

pam_status launch_interface_jump(pam_ctx *ctx, int n_fields, const pam_field *fields,
                                 const pam_dict *dict, const double *beta, int n, double *out) {
    std::vector<FaceDev> faces;
    for (int f = 0; f < n_fields; ++f) {
        const pam_field &F = fields[f];
        int ns[3] = {1, 1, 1}, off[3] = {0, 0, 0};
        for (int d = 0; d < F.dim; ++d) {
            ns[d] = F.n_sub_axis[d];
            if (d > 0) off[d] = off[d - 1] + F.n_sub_axis[d - 1] + 1;
        }
        const int tot = ns[0] * ns[1] * ns[2];
        const int stride[3] = {1, ns[0], ns[0] * ns[1]};
        for (int a = 0; a < F.dim; ++a) {
            for (int B = 0; B < tot; ++B) {
                const int kk[3] = {B % ns[0], (B / ns[0]) % ns[1], B / (ns[0] * ns[1])};
                if (kk[a] == 0) continue;
                FaceDev fc{};
                fc.a_sub = F.sub_base + B - stride[a];
                fc.b_sub = F.sub_base + B;
                fc.axis = a;
                fc.dim = F.dim;
                for (int d = 0; d < F.dim; ++d) {
                    fc.lo[d] = F.axis_x[off[d] + kk[d]];
                    fc.hi[d] = F.axis_x[off[d] + kk[d] + 1];
                }
                faces.push_back(fc);
            }
        }
    }
    if (faces.empty()) return PAM_OK;
    const size_t bytes = sizeof(FaceDev) * faces.size();
    pam_status st = ensure(ctx, BUF_EVAL, bytes);
    if (st != PAM_OK) return st;
    FaceDev *dfaces = wsp<FaceDev>(ctx, BUF_EVAL);
    if ((st = upload_to(ctx, dfaces, faces.data(), bytes)) != PAM_OK) return st;
    KernelTimer kt(ctx, PAM_TK_JUMP);
    hipLaunchKernelGGL(k_jump, dim3((unsigned)faces.size()), dim3(kJT), 0, ctx->stream, dfaces,
                       (int)faces.size(), n, dict->m_cap, dict->m, dict->c, dict->sigma, beta, out,
                       dict->basis == PAM_BASIS_PLAIN);
    PAM_CHECK_HIP(hipGetLastError());
    return PAM_OK;
}

}  // namespace pam
