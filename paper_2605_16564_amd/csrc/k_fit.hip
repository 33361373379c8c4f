// Per-subdomain fit kernels for gfx950: Shepard-normalized Gaussian design,
// MFMA Gram products, and the elastic-net solve (CD warm-up + exact
// sign-consistent active-set finish in FP64 with a KKT certificate).
//
// Paper steps: Eq. (gaussian_rbf) and Sec. 2 Step 2 (design at the samples),
// Def. 1 / Eq. (shepard_rbf) (row normalization), Eq. (elastic) and Sec. 3.3
// (elastic net by coordinate descent).
#include <float.h>
#include <hip/hip_bf16.h>

#include "pam_internal.h"

namespace pam {

static constexpr int kThreads = 256;
static constexpr int kWaves = kThreads / 64;
static constexpr int kChunk = 256;   // centers staged in LDS per pass

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double block_sum(double v, double *red) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    v = wave_sum(v);
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) r += red[w];
    __syncthreads();
    return r;
}

// Max of (value, index) with the lowest index winning ties.
struct VI { double v; int i; };
__device__ __forceinline__ VI better_max(VI a, VI b) {
    if (b.i < 0) return a;
    if (a.i < 0) return b;
    if (b.v > a.v) return b;
    if (b.v == a.v && b.i < a.i) return b;
    return a;
}
__device__ __forceinline__ VI block_argmax(VI x, double *redv, int *redi) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        VI y;
        y.v = __shfl_xor(x.v, o, 64);
        y.i = __shfl_xor(x.i, o, 64);
        x = better_max(x, y);
    }
    if (lane == 0) { redv[wid] = x.v; redi[wid] = x.i; }
    __syncthreads();
    VI r; r.v = -1.0; r.i = -1;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) { VI y; y.v = redv[w]; y.i = redi[w]; r = better_max(r, y); }
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_max(double v, double *redv, int *redi) {
    VI x; x.v = v; x.i = threadIdx.x;
    return block_argmax(x, redv, redi).v;
}

__device__ __forceinline__ double sgn(double v) { return v > 0.0 ? 1.0 : (v < 0.0 ? -1.0 : 0.0); }

// ---------------------------------------------------------------- assembly
// One thread per sample row j of subdomain s: pass 1 accumulates the Shepard
// denominator sum_m phi_m(x_j), pass 2 writes W_jm = phi_m(x_j)/sum into the
// transposed design Wt[m][j]; row M of Wt carries the data y so that the Gram
// product also yields b = W'y. Columns j >= N are zero padding.
template <typename TW>
__device__ __forceinline__ TW to_w(double v);
template <> __device__ __forceinline__ double to_w<double>(double v) { return v; }
template <> __device__ __forceinline__ float to_w<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ __hip_bfloat16 to_w<__hip_bfloat16>(double v) {
    return __float2bfloat16((float)v);
}

template <typename TW, bool kF64>
__global__ void __launch_bounds__(kThreads)
k_assemble(FitArgs a, TW *__restrict__ Wt, int32_t *__restrict__ flags) {
    const int s = a.sub_begin + blockIdx.y;
    if (a.active && !a.active[s]) return;
    const int64_t j0 = a.off[s];
    const int N = (int)(a.off[s + 1] - j0);
    const int M = max(0, min(a.m[s], a.m_cap));
    const int dim = a.dim;
    const int j = blockIdx.x * kThreads + threadIdx.x;
    __shared__ double sc[kChunk * 3];
    __shared__ double sa[kChunk];
    TW *W = Wt + (size_t)(s - a.sub_begin) * a.mpad * a.npad;
    double xj[3] = {0.0, 0.0, 0.0};
    const bool live = j < N;
    if (live)
        for (int d = 0; d < dim; ++d) xj[d] = a.x[(j0 + j) * dim + d];
    const double *cs = a.c + (size_t)s * a.m_cap * dim;
    const double *ss = a.sigma + (size_t)s * a.m_cap;
    double sum = 0.0;
    float sumf = 0.0f;
    for (int pass = 0; pass < 2; ++pass) {
        double inv = 0.0;
        float invf = 0.0f;
        if (pass == 1) {
            if (kF64) {
                if (live && !(sum >= DBL_MIN)) atomicOr(&flags[s], 1);
                inv = 1.0 / sum;
            } else {
                if (live && !(sumf >= FLT_MIN)) atomicOr(&flags[s], 1);
                invf = 1.0f / sumf;
            }
        }
        for (int m0 = 0; m0 < M; m0 += kChunk) {
            const int cnt = min(kChunk, M - m0);
            __syncthreads();
            for (int t = threadIdx.x; t < cnt; t += kThreads) {
                for (int d = 0; d < dim; ++d) sc[t * 3 + d] = cs[(size_t)(m0 + t) * dim + d];
                const double sg = ss[m0 + t];
                sa[t] = kF64 ? 0.5 / (sg * sg) : 1.4426950408889634 * 0.5 / (sg * sg);
            }
            __syncthreads();
            if (j < a.npad) {
                for (int t = 0; t < cnt; ++t) {
                    double r2 = 0.0;
                    for (int d = 0; d < dim; ++d) {
                        const double df = xj[d] - sc[t * 3 + d];
                        r2 += df * df;
                    }
                    if (kF64) {
                        const double p = exp(-r2 * sa[t]);
                        if (pass == 0) sum += p;
                        else W[(size_t)(m0 + t) * a.npad + j] = to_w<TW>(live ? p * inv : 0.0);
                    } else {
                        const float p = __builtin_amdgcn_exp2f(-(float)(r2 * sa[t]));
                        if (pass == 0) sumf += p;
                        else W[(size_t)(m0 + t) * a.npad + j] = to_w<TW>(live ? (double)(p * invf) : 0.0);
                    }
                }
            }
        }
    }
    if (j < a.npad) W[(size_t)M * a.npad + j] = to_w<TW>(live ? a.y[j0 + j] : 0.0);
}

// ---------------------------------------------------------------- Gram (MFMA)
// G = Wt Wt' over the (M+1) rows (basis rows and the data row), upper
// triangle of 64x64 tiles, mirrored into the lower triangle. Block of four
// waves; each wave owns a 32x32 quarter as 2x2 16x16 MFMA tiles. K (the
// sample index) is staged through LDS in chunks of 16.
typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void tile_of(int L, int nt, int &ti, int &tj) {
    // upper-triangular row-major enumeration: row ti holds nt - ti tiles
    ti = 0;
    while (L >= nt - ti) { L -= nt - ti; ++ti; }
    tj = ti + L;
}

__global__ void __launch_bounds__(kThreads)
k_gram_f64(FitArgs a, const double *__restrict__ Wt, double *__restrict__ G) {
    const int s = a.sub_begin + blockIdx.y;
    if (a.active && !a.active[s]) return;
    const int M1 = max(0, min(a.m[s], a.m_cap)) + 1;
    const int nt = (M1 + 63) / 64;
    if ((int)blockIdx.x >= nt * (nt + 1) / 2) return;
    int ti, tj;
    tile_of(blockIdx.x, nt, ti, tj);
    const int N = (int)(a.off[s + 1] - a.off[s]);
    const int Nk = (N + 15) & ~15;
    const double *W = Wt + (size_t)(s - a.sub_begin) * a.mpad * a.npad;
    double *Gs = G + (size_t)(s - a.sub_begin) * a.mpad * a.mpad;
    __shared__ double sA[64][17];
    __shared__ double sB[64][17];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int wr = wid >> 1, wc = wid & 1;
    const int m0 = ti * 64, n0 = tj * 64;
    v4d acc[2][2];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[p][q] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < Nk; k0 += 16) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = threadIdx.x + e * kThreads;  // 0..1023
            const int r = idx >> 4, cc = idx & 15;
            sA[r][cc] = W[(size_t)(m0 + r) * a.npad + k0 + cc];
            sB[r][cc] = W[(size_t)(n0 + r) * a.npad + k0 + cc];
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int kk = ks * 4 + (lane >> 4);
            double av[2], bv[2];
#pragma unroll
            for (int p = 0; p < 2; ++p) av[p] = sA[wr * 32 + p * 16 + (lane & 15)][kk];
#pragma unroll
            for (int q = 0; q < 2; ++q) bv[q] = sB[wc * 32 + q * 16 + (lane & 15)][kk];
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[p], bv[q], acc[p][q], 0, 0, 0);
        }
    }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                // FP64 16x16x4 output layout: lane l, register r -> (l/16 + 4r, l%16)
                const int row = m0 + wr * 32 + p * 16 + (lane >> 4) + 4 * r;
                const int col = n0 + wc * 32 + q * 16 + (lane & 15);
                Gs[(size_t)row * a.mpad + col] = acc[p][q][r];
                if (ti != tj) Gs[(size_t)col * a.mpad + row] = acc[p][q][r];
            }
}

// ---------------------------------------------------------------- solve
// One block per subdomain. Workspace per subdomain (global, L2 resident):
//   H [m_cap][m_cap]  inverse of (G + lambda2 I) on the active set, in
//                     active-list order, kept by bordering / Schur updates;
//   vec[0] g   gradient b - (G + lambda2 I) beta (full after consistent solves)
//   vec[1] beta
//   vec[2] z   solution of the reduced system (by active position)
//   vec[3] rhs (by active position)
//   vec[4] u / scratch (by active position)
//   vec[5] a   gathered column (by active position)
//   ivec[0] S  active list, ivec[1] pos (position or -1), ivec[2] theta
struct SolveWs {
    double *H, *vec;
    int32_t *ivec;
};

struct SubView {
    const double *G;   // [mpad][mpad]
    int mpad, M, m_cap;
    double l1, l2;
    double *H, *g, *beta, *z, *rhs, *u, *av;
    int *S, *pos, *th;
};

__device__ __forceinline__ double Gat(const SubView &v, int i, int j) {
    return v.G[(size_t)i * v.mpad + j];
}

// out_i = sum_j H[j][i] in_j for i < s (H symmetric; rows read coalesced).
// Blocks of 2048 outputs per pass keep the accumulators in registers.
__device__ void h_gemv(const SubView &v, int s, const double *in, double *out) {
    for (int base = 0; base < s; base += 8 * kThreads) {
        double acc[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) acc[r] = 0.0;
        const int lim = min(s - base, 8 * kThreads);
        for (int jj = 0; jj < s; ++jj) {
            const double x = in[jj];
            const double *Hr = v.H + (size_t)jj * v.m_cap + base;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int i = threadIdx.x + r * kThreads;
                if (i < lim) acc[r] += Hr[i] * x;
            }
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int i = threadIdx.x + r * kThreads;
            if (i < lim) out[base + i] = acc[r];
        }
    }
    __syncthreads();
}

// Append coordinate k to the active set: a = A[S,k], u = H a,
// delta = A_kk - a'u, H <- [[H + u u'/delta, -u/delta], [-u'/delta, 1/delta]].
// Returns false (and leaves the set unchanged) if delta is not positive.
__device__ bool fss_add(SubView &v, int &s, int k, double *red) {
    for (int i = threadIdx.x; i < s; i += kThreads) v.av[i] = Gat(v, k, v.S[i]);
    __syncthreads();
    h_gemv(v, s, v.av, v.u);
    double part = 0.0;
    for (int i = threadIdx.x; i < s; i += kThreads) part += v.av[i] * v.u[i];
    const double akk = Gat(v, k, k) + v.l2;
    const double delta = akk - block_sum(part, red);
    if (!(delta > 1e-14 * akk)) return false;
    const double id = 1.0 / delta;
    const int n1 = s + 1;
    for (int e = threadIdx.x; e < n1 * n1; e += kThreads) {
        const int i = e / n1, j = e - i * n1;
        double *p = v.H + (size_t)i * v.m_cap + j;
        if (i < s && j < s) *p += v.u[i] * v.u[j] * id;
        else if (i < s) *p = -v.u[i] * id;
        else if (j < s) *p = -v.u[j] * id;
        else *p = id;
    }
    if (threadIdx.x == 0) {
        v.S[s] = k;
        v.pos[k] = s;
    }
    __syncthreads();
    ++s;
    return true;
}

// Remove the coordinate at active position p: Schur downdate
// H <- H_{-p,-p} - h h' / H_pp with h = H[-p, p], then the last position is
// moved into p.
__device__ void fss_remove(SubView &v, int &s, int p) {
    const double hp = v.H[(size_t)p * v.m_cap + p];
    for (int i = threadIdx.x; i < s; i += kThreads) v.u[i] = v.H[(size_t)i * v.m_cap + p];
    __syncthreads();
    const double ih = 1.0 / hp;
    for (int e = threadIdx.x; e < s * s; e += kThreads) {
        const int i = e / s, j = e - i * s;
        if (i != p && j != p) v.H[(size_t)i * v.m_cap + j] -= v.u[i] * v.u[j] * ih;
    }
    __syncthreads();
    const int last = s - 1;
    const int kp = v.S[p];
    if (p != last) {
        for (int j = threadIdx.x; j < last; j += kThreads) {
            if (j == p) continue;
            const double val = v.H[(size_t)last * v.m_cap + j];
            v.H[(size_t)p * v.m_cap + j] = val;
            v.H[(size_t)j * v.m_cap + p] = val;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            v.H[(size_t)p * v.m_cap + p] = v.H[(size_t)last * v.m_cap + last];
            const int kl = v.S[last];
            v.S[p] = kl;
            v.pos[kl] = p;
        }
    }
    if (threadIdx.x == 0) v.pos[kp] = -1;
    __syncthreads();
    --s;
}

// Full gradient g = b - G beta - lambda2 beta over all M coordinates using the
// rows of the active coordinates (coalesced over m).
__device__ void full_gradient(SubView &v, int s) {
    for (int m = threadIdx.x; m < v.M; m += kThreads) {
        double acc = Gat(v, m, v.M);  // b_m (data column)
        for (int i = 0; i < s; ++i) {
            const int k = v.S[i];
            acc -= v.G[(size_t)k * v.mpad + m] * v.beta[k];
        }
        v.g[m] = acc - v.l2 * v.beta[m];
    }
    __syncthreads();
}

__global__ void __launch_bounds__(kThreads)
k_solve(FitArgs a, const double *__restrict__ Gall, SolveWs w, const int32_t *__restrict__ flags) {
    const int s_id = a.sub_begin + blockIdx.x;
    if (a.active && !a.active[s_id]) return;
    __shared__ double red[kWaves + 2];
    __shared__ double redv[kWaves];
    __shared__ int redi[kWaves];
    __shared__ int sh_flag;
    const int loc = s_id - a.sub_begin;
    SubView v;
    v.G = Gall + (size_t)loc * a.mpad * a.mpad;
    v.mpad = a.mpad;
    v.M = max(0, min(a.m[s_id], a.m_cap));
    v.m_cap = a.m_cap;
    v.l1 = a.lambda1_sub ? a.lambda1_sub[s_id] : a.lambda1;
    v.l2 = a.lambda2_sub ? a.lambda2_sub[s_id] : a.lambda2;
    v.H = w.H + (size_t)loc * a.m_cap * a.m_cap;
    double *vb = w.vec + (size_t)loc * 8 * a.m_cap;
    v.g = vb;
    v.beta = vb + a.m_cap;
    v.z = vb + 2 * a.m_cap;
    v.rhs = vb + 3 * a.m_cap;
    v.u = vb + 4 * a.m_cap;
    v.av = vb + 5 * a.m_cap;
    int32_t *ib = w.ivec + (size_t)loc * 3 * a.m_cap;
    v.S = ib;
    v.pos = ib + a.m_cap;
    v.th = ib + 2 * a.m_cap;
    const int M = v.M;
    double *beta_out = a.beta + (size_t)s_id * a.m_cap;
    pam_fit_stats *st = a.stats ? a.stats + s_id : nullptr;

    if (flags[s_id] & 1 || M <= 0 || a.off[s_id + 1] <= a.off[s_id]) {
        for (int m = threadIdx.x; m < a.m_cap; m += kThreads) beta_out[m] = 0.0;
        if (st && threadIdx.x == 0) {
            st->status = (flags[s_id] & 1) ? PAM_ST_UNDERFLOW : PAM_ST_EMPTY;
            st->cd_sweeps = 0; st->iters = 0; st->support = 0; st->kkt = 0.0;
        }
        return;
    }
    // ---- start point and gradient
    for (int m = threadIdx.x; m < M; m += kThreads) {
        v.beta[m] = a.warm_start ? beta_out[m] : 0.0;
        v.pos[m] = -1;
    }
    __syncthreads();
    for (int m = threadIdx.x; m < M; m += kThreads) v.g[m] = Gat(v, m, M) - v.l2 * v.beta[m];
    __syncthreads();
    if (a.warm_start) {
        for (int k = 0; k < M; ++k) {
            const double bk = v.beta[k];
            if (bk == 0.0) continue;
            for (int m = threadIdx.x; m < M; m += kThreads) v.g[m] -= v.G[(size_t)k * v.mpad + m] * bk;
        }
        __syncthreads();
    }
    // ---- cyclic coordinate descent warm-up (Sec. 3.3), creation order
    int sweeps = 0;
    for (; sweeps < a.cd_sweeps; ++sweeps) {
        for (int m = 0; m < M; ++m) {
            const double amm = Gat(v, m, m) + v.l2;
            const double bm = v.beta[m];
            const double zz = v.g[m] + amm * bm;
            const double az = fabs(zz) - v.l1;
            const double nb = az > 0.0 ? sgn(zz) * az / amm : 0.0;
            const double d = nb - bm;
            if (d != 0.0) {
                __syncthreads();
                for (int k = threadIdx.x; k < M; k += kThreads) v.g[k] -= v.G[(size_t)m * v.mpad + k] * d;
                __syncthreads();
                if (threadIdx.x == 0) {
                    v.g[m] -= v.l2 * d;
                    v.beta[m] = nb;
                }
                __syncthreads();
            }
        }
    }
    // ---- active set from the warm start (and the support hint)
    const uint8_t *hint = a.hint ? a.hint + (size_t)s_id * a.m_cap : nullptr;
    for (int m = threadIdx.x; m < M; m += kThreads) {
        int t = (int)sgn(v.beta[m]);
        if (t == 0 && hint && hint[m]) t = (int)sgn(v.g[m]);
        v.th[m] = t;
    }
    __syncthreads();
    int s = 0;
    for (int m = 0; m < M; ++m) {
        if (v.th[m] == 0) continue;
        if (!fss_add(v, s, m, red)) {
            if (threadIdx.x == 0) { v.th[m] = 0; v.beta[m] = 0.0; }
            __syncthreads();
        }
    }
    // gradient consistent with the (possibly pruned) start point
    full_gradient(v, s);

    // ---- exact sign-consistent active-set iteration (feature-sign search)
    double bnorm = 0.0;
    {
        double part = 0.0;
        for (int m = threadIdx.x; m < M; m += kThreads) part = fmax(part, fabs(Gat(v, m, M)));
        bnorm = block_max(part, redv, redi);
    }
    const double viol_tol = v.l1 * (1.0 + 1e-12) + 1e-14 * bnorm;
    int it = 0, status = PAM_ST_NOCONV, refines = 0;
    bool skip_solve = false;
    while (it < a.max_iter) {
        ++it;
        if (s > 0 && !skip_solve) {
            for (int i = threadIdx.x; i < s; i += kThreads) {
                const int k = v.S[i];
                v.rhs[i] = Gat(v, k, M) - v.l1 * (double)v.th[k];
            }
            __syncthreads();
            h_gemv(v, s, v.rhs, v.z);  // z = H rhs
            if (threadIdx.x == 0) sh_flag = 1;
            __syncthreads();
            for (int i = threadIdx.x; i < s; i += kThreads)
                if ((int)sgn(v.z[i]) != v.th[v.S[i]]) sh_flag = 0;
            __syncthreads();
            const bool consistent = sh_flag != 0;
            __syncthreads();
            if (!consistent) {
                // discrete line search from beta_S to z over the zero crossings
                double p1 = 0.0, p2 = 0.0;
                for (int i = threadIdx.x; i < s; i += kThreads) {
                    const int k = v.S[i];
                    const double d = v.z[i] - v.beta[k];
                    p1 -= v.g[k] * d;
                    p2 += d * (v.g[k] - v.l1 * (double)v.th[k]);
                }
                const double c1 = block_sum(p1, red);
                const double c2 = block_sum(p2, red);
                // candidate t for active position ci; ci == s stands for t = 1
                VI best; best.v = -DBL_MAX; best.i = -1;
                for (int ci = threadIdx.x; ci <= s; ci += kThreads) {
                    double t = 1.0;
                    bool ok = true;
                    if (ci < s) {
                        const int k = v.S[ci];
                        const double b0 = v.beta[k], zi = v.z[ci];
                        ok = b0 != 0.0 && sgn(zi) != sgn(b0);
                        if (ok) {
                            t = b0 / (b0 - zi);
                            ok = t > 0.0 && t < 1.0;
                        }
                    }
                    if (!ok) continue;
                    double l1s = 0.0;
                    for (int q = 0; q < s; ++q) {
                        const double b0 = v.beta[v.S[q]];
                        l1s += fabs(b0 + t * (v.z[q] - b0)) - fabs(b0);
                    }
                    const double f = t * c1 + 0.5 * t * t * c2 + v.l1 * l1s;
                    VI cand; cand.v = -f; cand.i = ci;
                    best = better_max(best, cand);
                }
                best = block_argmax(best, redv, redi);
                const int bi = best.i;
                double tstar = 1.0;
                if (bi >= 0 && bi < s) {
                    const int k = v.S[bi];
                    tstar = v.beta[k] / (v.beta[k] - v.z[bi]);
                }
                __syncthreads();
                for (int i = threadIdx.x; i < s; i += kThreads) {
                    const int k = v.S[i];
                    const double b0 = v.beta[k], zi = v.z[i];
                    double nb = b0 + tstar * (zi - b0);
                    if (tstar < 1.0 && b0 != 0.0 && sgn(zi) != sgn(b0) && b0 / (b0 - zi) == tstar) nb = 0.0;
                    v.g[k] -= tstar * (v.g[k] - v.l1 * (double)v.th[k]);
                    v.beta[k] = nb;
                    v.th[k] = (int)sgn(nb);
                }
                __syncthreads();
                for (int p = s - 1; p >= 0; --p) {
                    if (v.th[v.S[p]] == 0) fss_remove(v, s, p);
                }
                continue;
            }
            for (int i = threadIdx.x; i < s; i += kThreads) v.beta[v.S[i]] = v.z[i];
            __syncthreads();
        }
        skip_solve = false;
        full_gradient(v, s);
        // worst inactive violation
        VI x; x.v = -1.0; x.i = -1;
        for (int m = threadIdx.x; m < M; m += kThreads) {
            if (v.pos[m] >= 0) continue;
            VI c; c.v = fabs(v.g[m]); c.i = m;
            x = better_max(x, c);
        }
        x = block_argmax(x, redv, redi);
        if (x.i >= 0 && x.v > viol_tol) {
            // activate the worst violator with the descent sign
            const int k = x.i;
            if (threadIdx.x == 0) v.th[k] = (int)sgn(v.g[k]);
            __syncthreads();
            if (!fss_add(v, s, k, red)) break;
            continue;
        }
        // optimal up to the reduced-system residual r_S = g_S - lambda1 theta_S
        double rp = 0.0;
        for (int i = threadIdx.x; i < s; i += kThreads) {
            const int k = v.S[i];
            v.rhs[i] = v.g[k] - v.l1 * (double)v.th[k];
            rp = fmax(rp, fabs(v.rhs[i]));
        }
        const double rmax = block_max(rp, redv, redi);
        if (s == 0 || rmax <= 1e-15 * fmax(1.0, bnorm) || refines >= 3) {
            status = PAM_ST_OK;
            break;
        }
        ++refines;
        h_gemv(v, s, v.rhs, v.z);  // correction H r
        if (threadIdx.x == 0) sh_flag = 1;
        __syncthreads();
        for (int i = threadIdx.x; i < s; i += kThreads) {
            const int k = v.S[i];
            const double nb = v.beta[k] + v.z[i];
            if ((int)sgn(nb) != v.th[k]) sh_flag = 0;
        }
        __syncthreads();
        const bool keep = sh_flag != 0;
        __syncthreads();
        if (keep) {
            for (int i = threadIdx.x; i < s; i += kThreads) v.beta[v.S[i]] += v.z[i];
            __syncthreads();
            skip_solve = true;  // re-check the refined point without re-solving
        }
    }
    // ---- outputs and KKT residual (g is the full gradient here)
    __syncthreads();
    full_gradient(v, s);
    double kk = 0.0;
    int nz = 0;
    for (int m = threadIdx.x; m < M; m += kThreads) {
        const double b = v.beta[m];
        const double e = b != 0.0 ? fabs(v.g[m] - v.l1 * sgn(b)) : fmax(fabs(v.g[m]) - v.l1, 0.0);
        kk = fmax(kk, e);
        nz += b != 0.0;
    }
    const double kkt = block_max(kk, redv, redi);
    const double nzs = block_sum((double)nz, red);
    for (int m = threadIdx.x; m < a.m_cap; m += kThreads) beta_out[m] = m < M ? v.beta[m] : 0.0;
    if (st && threadIdx.x == 0) {
        st->status = status;
        st->cd_sweeps = sweeps;
        st->iters = it;
        st->support = (int)nzs;
        st->kkt = kkt;
    }
}

// ---------------------------------------------------------------- launchers
pam_status launch_assemble(pam_ctx *ctx, const FitArgs &a) {
    dim3 grid((a.npad + kThreads - 1) / kThreads, a.sub_count);
    int32_t *flags = wsp<int32_t>(ctx, BUF_FLAGS);
    if (a.precision == PAM_PREC_F64)
        hipLaunchKernelGGL((k_assemble<double, true>), grid, dim3(kThreads), 0, ctx->stream, a,
                           wsp<double>(ctx, BUF_WT), flags);
    else if (a.precision == PAM_PREC_F32)
        hipLaunchKernelGGL((k_assemble<float, false>), grid, dim3(kThreads), 0, ctx->stream, a,
                           wsp<float>(ctx, BUF_WT), flags);
    else
        hipLaunchKernelGGL((k_assemble<__hip_bfloat16, false>), grid, dim3(kThreads), 0, ctx->stream,
                           a, wsp<__hip_bfloat16>(ctx, BUF_WT), flags);
    PAM_CHECK_HIP(hipGetLastError());
    return PAM_OK;
}

pam_status launch_gram(pam_ctx *ctx, const FitArgs &a) {
    const int nt = a.mpad / 64;
    dim3 grid(nt * (nt + 1) / 2, a.sub_count);
    if (a.precision == PAM_PREC_F64) {
        hipLaunchKernelGGL(k_gram_f64, grid, dim3(kThreads), 0, ctx->stream, a,
                           wsp<double>(ctx, BUF_WT), wsp<double>(ctx, BUF_G));
    } else {
        set_error("Gram precision not available in this build");
        return PAM_ERR_ARG;
    }
    PAM_CHECK_HIP(hipGetLastError());
    return PAM_OK;
}

pam_status launch_solve(pam_ctx *ctx, const FitArgs &a) {
    SolveWs w;
    w.H = wsp<double>(ctx, BUF_H);
    w.vec = wsp<double>(ctx, BUF_VEC);
    w.ivec = wsp<int32_t>(ctx, BUF_IVEC);
    hipLaunchKernelGGL(k_solve, dim3(a.sub_count), dim3(kThreads), 0, ctx->stream, a,
                       wsp<double>(ctx, BUF_G), w, wsp<int32_t>(ctx, BUF_FLAGS));
    PAM_CHECK_HIP(hipGetLastError());
    return PAM_OK;
}

}  // namespace pam
