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
static constexpr int kChunk = 256;   // centers staged in LDS per pass

// ---------------------------------------------------------------- assembly
// One thread per sample row j of subdomain s: pass 1 accumulates the Shepard
// denominator sum_m phi_m(x_j), pass 2 writes W_jm = phi_m(x_j)/sum into the
// transposed design Wt[m][j]; row M of Wt carries the data y so that the Gram
// product also yields b = W'y. Columns j >= N are zero padding. The plain
// (unnormalized) basis skips pass 1 and writes phi_m(x_j) itself.
template <typename TW>
__device__ __forceinline__ TW to_w(double v);
template <> __device__ __forceinline__ double to_w<double>(double v) { return v; }
template <> __device__ __forceinline__ float to_w<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ __hip_bfloat16 to_w<__hip_bfloat16>(double v) {
    return __float2bfloat16((float)v);
}

// Input check (one block per subdomain): every sample coordinate, data value
// and element extent, and the first m[s] centers and widths must be finite,
// the widths positive. A failing subdomain is flagged (bit 2) so that the
// assembly, the solve and the marking skip it, and counted in the context's
// sticky word that pam_sync reports.
__global__ void __launch_bounds__(kThreads)
k_check_finite(FitArgs a, const double *__restrict__ h, int32_t *__restrict__ flags,
               int32_t *__restrict__ sticky) {
    const int s = blockIdx.x;
    if (a.active && !a.active[s]) return;
    const int64_t j0 = a.off[s];
    const int64_t nd = (a.off[s + 1] - j0) * a.dim;
    const int M = max(0, min(a.m[s], a.m_cap));
    int bad = 0;
    for (int64_t t = threadIdx.x; t < nd; t += kThreads) {
        bad |= !isfinite(a.x[j0 * a.dim + t]);
        if (h) bad |= !isfinite(h[j0 * a.dim + t]);
    }
    for (int64_t t = threadIdx.x; t < nd / a.dim; t += kThreads) bad |= !isfinite(a.y[j0 + t]);
    const double *cs = a.c + (size_t)s * a.m_cap * a.dim;
    const double *ss = a.sigma + (size_t)s * a.m_cap;
    for (int t = threadIdx.x; t < M * a.dim; t += kThreads) bad |= !isfinite(cs[t]);
    for (int t = threadIdx.x; t < M; t += kThreads) bad |= !(isfinite(ss[t]) && ss[t] > 0.0);
    if (__syncthreads_or(bad) && threadIdx.x == 0) {
        atomicOr(&flags[s], 2);
        atomicAdd(sticky, 1);
    }
}

pam_status launch_check_finite(pam_ctx *ctx, const FitArgs &a, const double *h) {
    hipLaunchKernelGGL(k_check_finite, dim3(a.n_sub), dim3(kThreads), 0, ctx->stream, a, h,
                       wsp<int32_t>(ctx, BUF_FLAGS), ctx->sticky);
    PAM_CHECK_HIP(hipGetLastError());
    return PAM_OK;
}

// Mask of the subdomains a refit serves: those whose last fit reported
// PAM_ST_NOCONV (stats of that fit, one entry per subdomain).
__global__ void __launch_bounds__(256)
k_noconv_mask(const pam_fit_stats *__restrict__ stats, int n, int32_t *__restrict__ mask) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s < n) mask[s] = stats[s].status == PAM_ST_NOCONV ? 1 : 0;
}

pam_status launch_noconv_mask(pam_ctx *ctx, const pam_fit_stats *stats, int n, int32_t *mask) {
    if (n <= 0) return PAM_OK;
    hipLaunchKernelGGL(k_noconv_mask, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, stats, n, mask);
    PAM_CHECK_HIP(hipGetLastError());
    return PAM_OK;
}

// One Gaussian of the low-precision modes: 2^(-(float)(r2 * sa)) with r2 the
// squared distance in FP64 and sa = log2(e) / (2 sigma^2). Contraction is off
// and the operations are written out once here, so that the assembly and the
// fused Gram (which recomputes the design inside its tiles) produce the same
// bits for every entry.
__device__ __forceinline__ double lp_scale(double sg) {
#pragma clang fp contract(off)
    return 0.7213475204444817 / (sg * sg);   // log2(e) / 2 / sigma^2
}
__device__ __forceinline__ float lp_phi(const double *x, const double *c, int dim, double sa) {
#pragma clang fp contract(off)
    double r2 = 0.0;
    for (int d = 0; d < dim; ++d) {
        const double df = x[d] - c[d];
        r2 = r2 + df * df;
    }
    return __builtin_amdgcn_exp2f(-(float)(r2 * sa));
}

template <typename TW, bool kF64>
__global__ void __launch_bounds__(kThreads)
k_assemble(FitArgs a, TW *__restrict__ Wt, int32_t *__restrict__ flags) {
    const int s = a.sub_begin + blockIdx.y;
    if (a.active && !a.active[s]) return;
    if (flags[s] & 2) return;   // non-finite input: not fitted
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
    for (int pass = a.basis == PAM_BASIS_PLAIN ? 1 : 0; pass < 2; ++pass) {
        double inv = 0.0;
        float invf = 0.0f;
        if (pass == 1 && a.basis == PAM_BASIS_PLAIN) {
            inv = 1.0;
            invf = 1.0f;
        } else if (pass == 1) {
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
                sa[t] = kF64 ? 0.5 / (sg * sg) : lp_scale(sg);
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
                        const float p = lp_phi(xj, &sc[t * 3], dim, sa[t]);
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

// FP32 and BF16 variants: FP32 accumulation, G stored as FP32. The 16x16
// output layout of these instructions is lane l, register r -> (4(l/16)+r, l%16).
__global__ void __launch_bounds__(kThreads)
k_gram_f32(FitArgs a, const float *__restrict__ Wt, float *__restrict__ G) {
    const int s = a.sub_begin + blockIdx.y;
    if (a.active && !a.active[s]) return;
    const int M1 = max(0, min(a.m[s], a.m_cap)) + 1;
    const int nt = (M1 + 63) / 64;
    if ((int)blockIdx.x >= nt * (nt + 1) / 2) return;
    int ti, tj;
    tile_of(blockIdx.x, nt, ti, tj);
    const int N = (int)(a.off[s + 1] - a.off[s]);
    const int Nk = (N + 15) & ~15;
    const float *W = Wt + (size_t)(s - a.sub_begin) * a.mpad * a.npad;
    float *Gs = G + (size_t)(s - a.sub_begin) * a.mpad * a.mpad;
    __shared__ float sA[64][17];
    __shared__ float sB[64][17];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int wr = wid >> 1, wc = wid & 1;
    const int m0 = ti * 64, n0 = tj * 64;
    v4f acc[2][2];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[p][q] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < Nk; k0 += 16) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = threadIdx.x + e * kThreads;
            const int r = idx >> 4, cc = idx & 15;
            sA[r][cc] = W[(size_t)(m0 + r) * a.npad + k0 + cc];
            sB[r][cc] = W[(size_t)(n0 + r) * a.npad + k0 + cc];
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int kk = ks * 4 + (lane >> 4);
            float av[2], bv[2];
#pragma unroll
            for (int p = 0; p < 2; ++p) av[p] = sA[wr * 32 + p * 16 + (lane & 15)][kk];
#pragma unroll
            for (int q = 0; q < 2; ++q) bv[q] = sB[wc * 32 + q * 16 + (lane & 15)][kk];
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    acc[p][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[p], bv[q], acc[p][q], 0, 0, 0);
        }
    }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wr * 32 + p * 16 + 4 * (lane >> 4) + r;
                const int col = n0 + wc * 32 + q * 16 + (lane & 15);
                Gs[(size_t)row * a.mpad + col] = acc[p][q][r];
                if (ti != tj) Gs[(size_t)col * a.mpad + row] = acc[p][q][r];
            }
}

__global__ void __launch_bounds__(kThreads)
k_gram_bf16(FitArgs a, const __hip_bfloat16 *__restrict__ Wt, float *__restrict__ G) {
    const int s = a.sub_begin + blockIdx.y;
    if (a.active && !a.active[s]) return;
    const int M1 = max(0, min(a.m[s], a.m_cap)) + 1;
    const int nt = (M1 + 63) / 64;
    if ((int)blockIdx.x >= nt * (nt + 1) / 2) return;
    int ti, tj;
    tile_of(blockIdx.x, nt, ti, tj);
    const int N = (int)(a.off[s + 1] - a.off[s]);
    const int Nk = (N + 31) & ~31;
    const unsigned short *W = reinterpret_cast<const unsigned short *>(Wt) +
                              (size_t)(s - a.sub_begin) * a.mpad * a.npad;
    float *Gs = G + (size_t)(s - a.sub_begin) * a.mpad * a.mpad;
    // rows of 32 bf16 (64 B) + 16 B pad to spread LDS banks
    __shared__ __attribute__((aligned(16))) unsigned short sA[64][40];
    __shared__ __attribute__((aligned(16))) unsigned short sB[64][40];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int wr = wid >> 1, wc = wid & 1;
    const int m0 = ti * 64, n0 = tj * 64;
    v4f acc[2][2];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[p][q] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < Nk; k0 += 32) {
        __syncthreads();
        {
            // 64 rows x 32 bf16 = 256 x 16-byte vectors per operand: one each per thread
            const int r = threadIdx.x >> 2, c8 = (threadIdx.x & 3) * 8;
            *reinterpret_cast<uint4 *>(&sA[r][c8]) =
                *reinterpret_cast<const uint4 *>(W + (size_t)(m0 + r) * a.npad + k0 + c8);
            *reinterpret_cast<uint4 *>(&sB[r][c8]) =
                *reinterpret_cast<const uint4 *>(W + (size_t)(n0 + r) * a.npad + k0 + c8);
        }
        __syncthreads();
        const int kb = 8 * (lane >> 4);
        v8bf av[2], bv[2];
#pragma unroll
        for (int p = 0; p < 2; ++p)
            av[p] = *reinterpret_cast<const v8bf *>(&sA[wr * 32 + p * 16 + (lane & 15)][kb]);
#pragma unroll
        for (int q = 0; q < 2; ++q)
            bv[q] = *reinterpret_cast<const v8bf *>(&sB[wc * 32 + q * 16 + (lane & 15)][kb]);
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < 2; ++q)
                acc[p][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[p], bv[q], acc[p][q], 0, 0, 0);
    }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wr * 32 + p * 16 + 4 * (lane >> 4) + r;
                const int col = n0 + wc * 32 + q * 16 + (lane & 15);
                Gs[(size_t)row * a.mpad + col] = acc[p][q][r];
                if (ti != tj) Gs[(size_t)col * a.mpad + row] = acc[p][q][r];
            }
}

// ---------------------------------------------------------------- fused path
// The low-precision design without its HBM round trip: k_rowsum computes the
// Shepard denominators exactly as the assembly's first pass (inv[j] =
// 1 / sum_m phi_jm, the same order of the same float sums), then the fused
// Gram tiles compute every W_mj = phi_mj * inv[j] they need in LDS and
// contract them on MFMA: the Gram is the same bits as through the stored
// design, and W never reaches HBM (at the price of recomputing each entry in
// every tile that uses it).
__global__ void __launch_bounds__(kThreads)
k_rowsum(FitArgs a, float *__restrict__ inv, int32_t *__restrict__ flags) {
    const int s = a.sub_begin + blockIdx.y;
    if (a.active && !a.active[s]) return;
    if (flags[s] & 2) return;
    const int64_t j0 = a.off[s];
    const int N = (int)(a.off[s + 1] - j0);
    const int M = max(0, min(a.m[s], a.m_cap));
    const int dim = a.dim;
    const int j = blockIdx.x * kThreads + threadIdx.x;
    __shared__ double sc[kChunk * 3];
    __shared__ double sa[kChunk];
    float *is = inv + (size_t)(s - a.sub_begin) * a.npad;
    const bool live = j < N;
    double xj[3] = {0.0, 0.0, 0.0};
    if (live)
        for (int d = 0; d < dim; ++d) xj[d] = a.x[(j0 + j) * dim + d];
    if (a.basis == PAM_BASIS_PLAIN) {
        if (j < a.npad) is[j] = 1.0f;
        return;
    }
    const double *cs = a.c + (size_t)s * a.m_cap * dim;
    const double *ss = a.sigma + (size_t)s * a.m_cap;
    float sumf = 0.0f;
    for (int m0 = 0; m0 < M; m0 += kChunk) {
        const int cnt = min(kChunk, M - m0);
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += kThreads) {
            for (int d = 0; d < dim; ++d) sc[t * 3 + d] = cs[(size_t)(m0 + t) * dim + d];
            sa[t] = lp_scale(ss[m0 + t]);
        }
        __syncthreads();
        if (live)
            for (int t = 0; t < cnt; ++t) sumf += lp_phi(xj, &sc[t * 3], dim, sa[t]);
    }
    if (live && !(sumf >= FLT_MIN)) atomicOr(&flags[s], 1);
    if (j < a.npad) is[j] = 1.0f / sumf;
}

// Value of the design entry (center row m, sample column j) as the assembly
// stores it: rows m < M the normalized Gaussians, row M the data, zero for
// padded samples and rows beyond M.
template <typename TW>
__device__ __forceinline__ TW fused_entry(int m, int M, bool live, const double *xj, const double *cm, int dim,
                                          double sa, float invf, double yj) {
    if (!live || m > M) return to_w<TW>(0.0);
    if (m == M) return to_w<TW>(yj);
    return to_w<TW>((double)(lp_phi(xj, cm, dim, sa) * invf));
}

template <typename TW, int KC>
struct FusedStage {
    double c[2][64][3];   // centers of the two tile rows
    double sa[2][64];
    double x[KC][3];      // the chunk's samples
    double y[KC];
    float inv[KC];
    int live[KC];
};

// Stage the two tiles' centers (rows m0.., n0..) once per block.
template <typename TW, int KC>
__device__ __forceinline__ void fused_centers(const FitArgs &a, int s, int M, int m0, int n0, FusedStage<TW, KC> &st) {
    const double *cs = a.c + (size_t)s * a.m_cap * a.dim;
    const double *ss = a.sigma + (size_t)s * a.m_cap;
    for (int t = threadIdx.x; t < 128; t += kThreads) {
        const int side = t >> 6, r = t & 63;
        const int m = (side ? n0 : m0) + r;
        for (int d = 0; d < 3; ++d) st.c[side][r][d] = (m < M && d < a.dim) ? cs[(size_t)m * a.dim + d] : 0.0;
        st.sa[side][r] = m < M ? lp_scale(ss[m]) : 0.0;
    }
}

template <typename TW, int KC>
__device__ __forceinline__ void fused_samples(const FitArgs &a, int64_t j0, int N, int k0, const float *is,
                                              FusedStage<TW, KC> &st) {
    for (int t = threadIdx.x; t < KC; t += kThreads) {
        const int j = k0 + t;
        const bool live = j < N;
        st.live[t] = live;
        for (int d = 0; d < 3; ++d) st.x[t][d] = (live && d < a.dim) ? a.x[(j0 + j) * a.dim + d] : 0.0;
        st.y[t] = live ? a.y[j0 + j] : 0.0;
        st.inv[t] = live ? is[j] : 0.0f;
    }
}

__global__ void __launch_bounds__(kThreads)
k_gram_fused_f32(FitArgs a, const float *__restrict__ inv, float *__restrict__ G, const int32_t *__restrict__ flags) {
    const int s = a.sub_begin + blockIdx.y;
    if (a.active && !a.active[s]) return;
    if (flags[s] & 2) return;
    const int M = max(0, min(a.m[s], a.m_cap));
    const int M1 = M + 1;
    const int nt = (M1 + 63) / 64;
    if ((int)blockIdx.x >= nt * (nt + 1) / 2) return;
    int ti, tj;
    tile_of(blockIdx.x, nt, ti, tj);
    const int64_t j0 = a.off[s];
    const int N = (int)(a.off[s + 1] - j0);
    const int Nk = (N + 15) & ~15;
    const float *is = inv + (size_t)(s - a.sub_begin) * a.npad;
    float *Gs = G + (size_t)(s - a.sub_begin) * a.mpad * a.mpad;
    __shared__ float sA[64][17];
    __shared__ float sB[64][17];
    __shared__ FusedStage<float, 16> st;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int wr = wid >> 1, wc = wid & 1;
    const int m0 = ti * 64, n0 = tj * 64;
    fused_centers<float, 16>(a, s, M, m0, n0, st);
    v4f acc[2][2];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[p][q] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < Nk; k0 += 16) {
        __syncthreads();
        fused_samples<float, 16>(a, j0, N, k0, is, st);
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = threadIdx.x + e * kThreads;
            const int r = idx >> 4, cc = idx & 15;
            const float va = fused_entry<float>(m0 + r, M, st.live[cc], st.x[cc], st.c[0][r], a.dim, st.sa[0][r],
                                                st.inv[cc], st.y[cc]);
            sA[r][cc] = va;
            sB[r][cc] = ti == tj ? va
                                 : fused_entry<float>(n0 + r, M, st.live[cc], st.x[cc], st.c[1][r], a.dim,
                                                      st.sa[1][r], st.inv[cc], st.y[cc]);
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int kk = ks * 4 + (lane >> 4);
            float av[2], bv[2];
#pragma unroll
            for (int p = 0; p < 2; ++p) av[p] = sA[wr * 32 + p * 16 + (lane & 15)][kk];
#pragma unroll
            for (int q = 0; q < 2; ++q) bv[q] = sB[wc * 32 + q * 16 + (lane & 15)][kk];
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    acc[p][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[p], bv[q], acc[p][q], 0, 0, 0);
        }
    }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wr * 32 + p * 16 + 4 * (lane >> 4) + r;
                const int col = n0 + wc * 32 + q * 16 + (lane & 15);
                Gs[(size_t)row * a.mpad + col] = acc[p][q][r];
                if (ti != tj) Gs[(size_t)col * a.mpad + row] = acc[p][q][r];
            }
}

__global__ void __launch_bounds__(kThreads)
k_gram_fused_bf16(FitArgs a, const float *__restrict__ inv, float *__restrict__ G, const int32_t *__restrict__ flags) {
    const int s = a.sub_begin + blockIdx.y;
    if (a.active && !a.active[s]) return;
    if (flags[s] & 2) return;
    const int M = max(0, min(a.m[s], a.m_cap));
    const int M1 = M + 1;
    const int nt = (M1 + 63) / 64;
    if ((int)blockIdx.x >= nt * (nt + 1) / 2) return;
    int ti, tj;
    tile_of(blockIdx.x, nt, ti, tj);
    const int64_t j0 = a.off[s];
    const int N = (int)(a.off[s + 1] - j0);
    const int Nk = (N + 31) & ~31;
    const float *is = inv + (size_t)(s - a.sub_begin) * a.npad;
    float *Gs = G + (size_t)(s - a.sub_begin) * a.mpad * a.mpad;
    __shared__ __attribute__((aligned(16))) __hip_bfloat16 sA[64][40];
    __shared__ __attribute__((aligned(16))) __hip_bfloat16 sB[64][40];
    __shared__ FusedStage<__hip_bfloat16, 32> st;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int wr = wid >> 1, wc = wid & 1;
    const int m0 = ti * 64, n0 = tj * 64;
    fused_centers<__hip_bfloat16, 32>(a, s, M, m0, n0, st);
    v4f acc[2][2];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[p][q] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < Nk; k0 += 32) {
        __syncthreads();
        fused_samples<__hip_bfloat16, 32>(a, j0, N, k0, is, st);
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int idx = threadIdx.x + e * kThreads;   // 0..2047
            const int r = idx >> 5, cc = idx & 31;
            const __hip_bfloat16 va = fused_entry<__hip_bfloat16>(m0 + r, M, st.live[cc], st.x[cc], st.c[0][r],
                                                                  a.dim, st.sa[0][r], st.inv[cc], st.y[cc]);
            sA[r][cc] = va;
            sB[r][cc] = ti == tj ? va
                                 : fused_entry<__hip_bfloat16>(n0 + r, M, st.live[cc], st.x[cc], st.c[1][r],
                                                               a.dim, st.sa[1][r], st.inv[cc], st.y[cc]);
        }
        __syncthreads();
        const int kb = 8 * (lane >> 4);
        v8bf av[2], bv[2];
#pragma unroll
        for (int p = 0; p < 2; ++p)
            av[p] = *reinterpret_cast<const v8bf *>(&sA[wr * 32 + p * 16 + (lane & 15)][kb]);
#pragma unroll
        for (int q = 0; q < 2; ++q)
            bv[q] = *reinterpret_cast<const v8bf *>(&sB[wc * 32 + q * 16 + (lane & 15)][kb]);
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < 2; ++q)
                acc[p][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[p], bv[q], acc[p][q], 0, 0, 0);
    }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wr * 32 + p * 16 + 4 * (lane >> 4) + r;
                const int col = n0 + wc * 32 + q * 16 + (lane & 15);
                Gs[(size_t)row * a.mpad + col] = acc[p][q][r];
                if (ti != tj) Gs[(size_t)col * a.mpad + row] = acc[p][q][r];
            }
}

// ---------------------------------------------------------------- launchers
pam_status launch_rowsum(pam_ctx *ctx, const FitArgs &a) {
    dim3 grid((a.npad + kThreads - 1) / kThreads, a.sub_count);
    hipLaunchKernelGGL(k_rowsum, grid, dim3(kThreads), 0, ctx->stream, a, wsp<float>(ctx, BUF_ROWSUM),
                       wsp<int32_t>(ctx, BUF_FLAGS));
    PAM_CHECK_HIP(hipGetLastError());
    return PAM_OK;
}

pam_status launch_gram_fused(pam_ctx *ctx, const FitArgs &a) {
    const int nt = a.mpad / 64;
    dim3 grid(nt * (nt + 1) / 2, a.sub_count);
    if (a.precision == PAM_PREC_F32)
        hipLaunchKernelGGL(k_gram_fused_f32, grid, dim3(kThreads), 0, ctx->stream, a, wsp<float>(ctx, BUF_ROWSUM),
                           wsp<float>(ctx, BUF_G), wsp<int32_t>(ctx, BUF_FLAGS));
    else
        hipLaunchKernelGGL(k_gram_fused_bf16, grid, dim3(kThreads), 0, ctx->stream, a,
                           wsp<float>(ctx, BUF_ROWSUM), wsp<float>(ctx, BUF_G), wsp<int32_t>(ctx, BUF_FLAGS));
    PAM_CHECK_HIP(hipGetLastError());
    return PAM_OK;
}

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
    if (a.precision == PAM_PREC_F64)
        hipLaunchKernelGGL(k_gram_f64, grid, dim3(kThreads), 0, ctx->stream, a,
                           wsp<double>(ctx, BUF_WT), wsp<double>(ctx, BUF_G));
    else if (a.precision == PAM_PREC_F32)
        hipLaunchKernelGGL(k_gram_f32, grid, dim3(kThreads), 0, ctx->stream, a,
                           wsp<float>(ctx, BUF_WT), wsp<float>(ctx, BUF_G));
    else
        hipLaunchKernelGGL(k_gram_bf16, grid, dim3(kThreads), 0, ctx->stream, a,
                           wsp<__hip_bfloat16>(ctx, BUF_WT), wsp<float>(ctx, BUF_G));
    PAM_CHECK_HIP(hipGetLastError());
    return PAM_OK;
}

}  // namespace pam
