// Darcy consumer of the reconstruction (Sec. 5, Eq. (darcy_model); the
// pressure experiment of Exp. 1): -div(K grad p) = 0 on a box, p = p_left on
// the left face, p = p_right on the right face, no flow across the others;
// continuous P1 elements on the n0 x n1 squares of the box, each split along
// its (i, j)-(i+1, j+1) diagonal, K constant per triangle.
//
// On these right triangles the element matrix has no coupling along the
// diagonal, so the operator is a five-point stencil on the nodes: a
// horizontal edge weighs hy / (2 hx) times the sum of K over the (one or two)
// triangles that own it, a vertical edge hx / (2 hy) times theirs, and
// (A p)_v = sum over edges (v, u) of w (p_v - p_u). Dirichlet nodes are
// eliminated (their rows are the identity, their values enter the residual),
// and the system is solved by Jacobi-preconditioned conjugate gradients in
// FP64. Scalars of the iteration stay on the device: every block sums the
// per-block partial products in the same fixed order, so all blocks agree.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "pam_internal.h"

namespace pam {

static constexpr int kD = 256;

struct DarcyDev {
    int n0, n1;          // squares per axis; nodes (n0 + 1) x (n1 + 1)
    double cx, cy;       // hy / (2 hx), hx / (2 hy)
    double p_left, p_right;
    const double *k;     // [n1][n0][2]: 0 lower-right, 1 upper-left
    double *wh;          // horizontal edge (i, j)-(i+1, j): [(n1 + 1)][n0]
    double *wv;          // vertical edge (i, j)-(i, j+1): [n1][(n0 + 1)]
    double *diag, *x, *r, *z, *d, *q;
    double *part;        // [3][nblk] per-block partial sums
    double *sc;          // [4]: rz (two slots, by iteration parity), rr, bb
    int nblk;
};

__device__ __forceinline__ bool is_dirichlet(const DarcyDev &D, int v) {
    const int i = v % (D.n0 + 1);
    return i == 0 || i == D.n0;
}

__device__ __forceinline__ double apply_row(const DarcyDev &D, const double *u, int v) {
    const int i = v % (D.n0 + 1), j = v / (D.n0 + 1);
    const double uv = u[v];
    double s = 0.0;
    if (i > 0) s += D.wh[j * D.n0 + i - 1] * (uv - u[v - 1]);
    if (i < D.n0) s += D.wh[j * D.n0 + i] * (uv - u[v + 1]);
    if (j > 0) s += D.wv[(j - 1) * (D.n0 + 1) + i] * (uv - u[v - (D.n0 + 1)]);
    if (j < D.n1) s += D.wv[j * (D.n0 + 1) + i] * (uv - u[v + (D.n0 + 1)]);
    return s;
}

// Sum of a block's values into part[slot][blockIdx] (fixed tree order).
__device__ __forceinline__ void block_partial(double v, double *red, double *dst) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int k = kD / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *dst = red[0];
    __syncthreads();
}

// Total of a partial array, the same order in every block.
__device__ __forceinline__ double total(const double *p, int n, double *red) {
    double s = 0.0;
    for (int b = threadIdx.x; b < n; b += kD) s += p[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = kD / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    const double t = red[0];
    __syncthreads();
    return t;
}

// Edge weights from the triangle values.
__global__ void __launch_bounds__(kD) k_darcy_edges(DarcyDev D) {
    const int e = blockIdx.x * kD + threadIdx.x;
    const int nh = (D.n1 + 1) * D.n0, nv = D.n1 * (D.n0 + 1);
    if (e < nh) {
        const int i = e % D.n0, j = e / D.n0;
        double s = 0.0;
        if (j < D.n1) s += D.k[((size_t)j * D.n0 + i) * 2 + 0];        // bottom edge of lower-right
        if (j > 0) s += D.k[((size_t)(j - 1) * D.n0 + i) * 2 + 1];    // top edge of upper-left
        D.wh[e] = D.cx * s;
    } else if (e < nh + nv) {
        const int f = e - nh;
        const int i = f % (D.n0 + 1), j = f / (D.n0 + 1);
        double s = 0.0;
        if (i < D.n0) s += D.k[((size_t)j * D.n0 + i) * 2 + 1];        // left edge of upper-left
        if (i > 0) s += D.k[((size_t)j * D.n0 + i - 1) * 2 + 0];      // right edge of lower-right
        D.wv[f] = D.cy * s;
    }
}

// Start: x linear between the Dirichlet values on free nodes (cold) and the
// Dirichlet values themselves (always).
__global__ void __launch_bounds__(kD) k_darcy_start(DarcyDev D, int warm) {
    const int N = (D.n0 + 1) * (D.n1 + 1);
    const int v = blockIdx.x * kD + threadIdx.x;
    if (v >= N) return;
    const int i = v % (D.n0 + 1);
    if (is_dirichlet(D, v))
        D.x[v] = i == 0 ? D.p_left : D.p_right;
    else if (!warm)
        D.x[v] = D.p_left + (D.p_right - D.p_left) * i / D.n0;
}

// Residual r = -A x on free nodes (0 on Dirichlet nodes), the Jacobi
// diagonal, z = r / diag, d = z; partials of r.z, r.r and b.b, where b (the
// right-hand side once the Dirichlet values are moved to it) is the sum of
// w p_D over a free node's edges to Dirichlet nodes.
__global__ void __launch_bounds__(kD) k_darcy_res(DarcyDev D) {
    __shared__ double red[kD];
    const int N = (D.n0 + 1) * (D.n1 + 1);
    const int v = blockIdx.x * kD + threadIdx.x;
    double rz = 0.0, rr = 0.0, bb = 0.0;
    if (v < N) {
        const int i = v % (D.n0 + 1), j = v / (D.n0 + 1);
        double dg = 0.0;
        if (i > 0) dg += D.wh[j * D.n0 + i - 1];
        if (i < D.n0) dg += D.wh[j * D.n0 + i];
        if (j > 0) dg += D.wv[(j - 1) * (D.n0 + 1) + i];
        if (j < D.n1) dg += D.wv[j * (D.n0 + 1) + i];
        D.diag[v] = dg;
        double r = 0.0, z = 0.0, b = 0.0;
        if (!is_dirichlet(D, v)) {
            r = -apply_row(D, D.x, v);
            z = dg > 0.0 ? r / dg : 0.0;
            if (i == 1) b += D.wh[j * D.n0] * D.p_left;
            if (i == D.n0 - 1) b += D.wh[j * D.n0 + D.n0 - 1] * D.p_right;
        }
        D.r[v] = r;
        D.z[v] = z;
        D.d[v] = z;
        rz = r * z;
        rr = r * r;
        bb = b * b;
    }
    block_partial(rz, red, &D.part[blockIdx.x]);
    block_partial(rr, red, &D.part[D.nblk + blockIdx.x]);
    block_partial(bb, red, &D.part[2 * D.nblk + blockIdx.x]);
}

// rz (slot 0), rr and bb from the start partials.
__global__ void __launch_bounds__(kD) k_darcy_init_scalars(DarcyDev D) {
    __shared__ double red[kD];
    const double rz = total(D.part, D.nblk, red);
    const double rr = total(D.part + D.nblk, D.nblk, red);
    const double bb = total(D.part + 2 * D.nblk, D.nblk, red);
    if (threadIdx.x == 0) {
        D.sc[0] = rz;
        D.sc[2] = rr;
        D.sc[3] = bb;
    }
}

// q = A d on free nodes (0 on Dirichlet nodes); partials of d.q.
__global__ void __launch_bounds__(kD) k_darcy_matvec(DarcyDev D) {
    __shared__ double red[kD];
    const int N = (D.n0 + 1) * (D.n1 + 1);
    const int v = blockIdx.x * kD + threadIdx.x;
    double dq = 0.0;
    if (v < N) {
        const double q = is_dirichlet(D, v) ? 0.0 : apply_row(D, D.d, v);
        D.q[v] = q;
        dq = D.d[v] * q;
    }
    block_partial(dq, red, &D.part[2 * D.nblk + blockIdx.x]);
}

// alpha = rz / d.q; x += alpha d; r -= alpha q; z = r / diag; partials of
// the new r.z and r.r.
__global__ void __launch_bounds__(kD) k_darcy_update(DarcyDev D, int par) {
    __shared__ double red[kD];
    const int N = (D.n0 + 1) * (D.n1 + 1);
    const double dq = total(D.part + 2 * D.nblk, D.nblk, red);
    const double rz = D.sc[par];
    const double alpha = dq > 0.0 ? rz / dq : 0.0;
    const int v = blockIdx.x * kD + threadIdx.x;
    double rzn = 0.0, rr = 0.0;
    if (v < N) {
        D.x[v] += alpha * D.d[v];
        const double r = D.r[v] - alpha * D.q[v];
        const double dg = D.diag[v];
        const double z = is_dirichlet(D, v) || !(dg > 0.0) ? 0.0 : r / dg;
        D.r[v] = r;
        D.z[v] = z;
        rzn = r * z;
        rr = r * r;
    }
    block_partial(rzn, red, &D.part[blockIdx.x]);
    block_partial(rr, red, &D.part[D.nblk + blockIdx.x]);
}

// beta = rz_new / rz; d = z + beta d; rz_new into the other slot; rr.
__global__ void __launch_bounds__(kD) k_darcy_direction(DarcyDev D, int par) {
    __shared__ double red[kD];
    const int N = (D.n0 + 1) * (D.n1 + 1);
    const double rzn = total(D.part, D.nblk, red);
    const double rr = total(D.part + D.nblk, D.nblk, red);
    const double rz = D.sc[par];
    const double beta = rz > 0.0 ? rzn / rz : 0.0;
    const int v = blockIdx.x * kD + threadIdx.x;
    if (v < N) D.d[v] = D.z[v] + beta * D.d[v];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        D.sc[1 - par] = rzn;
        D.sc[2] = rr;
    }
}

// Per-block partials of the P1 L2 products of e = a - b and of a:
// |T| / 12 (sum u^2 + (sum u)^2) per triangle.
__global__ void __launch_bounds__(kD)
k_darcy_norms(int n0, int n1, double area, const double *__restrict__ a,
              const double *__restrict__ b, double *__restrict__ part, int nblk) {
    __shared__ double red[kD];
    const int t = blockIdx.x * kD + threadIdx.x;
    double ee = 0.0, aa = 0.0;
    if (t < 2 * n0 * n1) {
        const int sq = t / 2, i = sq % n0, j = sq / n0;
        const int v00 = j * (n0 + 1) + i, v10 = v00 + 1, v01 = v00 + n0 + 1, v11 = v01 + 1;
        const int w0 = v00, w1 = (t % 2 == 0) ? v10 : v11, w2 = (t % 2 == 0) ? v11 : v01;
        const double e0 = a[w0] - b[w0], e1 = a[w1] - b[w1], e2 = a[w2] - b[w2];
        const double se = e0 + e1 + e2;
        ee = area / 12.0 * (e0 * e0 + e1 * e1 + e2 * e2 + se * se);
        const double a0 = a[w0], a1 = a[w1], a2 = a[w2];
        const double sa = a0 + a1 + a2;
        aa = area / 12.0 * (a0 * a0 + a1 * a1 + a2 * a2 + sa * sa);
    }
    block_partial(ee, red, &part[blockIdx.x]);
    block_partial(aa, red, &part[nblk + blockIdx.x]);
}

__global__ void __launch_bounds__(kD)
k_darcy_norms_total(const double *__restrict__ part, int nblk, double *__restrict__ out) {
    __shared__ double red[kD];
    const double ee = total(part, nblk, red);
    const double aa = total(part + nblk, nblk, red);
    if (threadIdx.x == 0) {
        out[0] = ee;
        out[1] = aa;
    }
}

// ---------------------------------------------------------------- launchers
// A burst of `len` iterations (three kernels each, iteration b with parity
// (par0 + b) & 1) as one executable graph: a chain of kernel nodes with the
// arguments baked in, launched once per convergence check instead of 3 len
// separate launches (the stencil pass itself is a few microseconds).
static pam_status build_burst(const DarcyDev &D, int len, int par0, hipGraphExec_t *exec) {
    hipGraph_t g = nullptr;
    PAM_CHECK_HIP(hipGraphCreate(&g, 0));
    hipError_t e = hipSuccess;
    hipGraphNode_t prev = nullptr;
    DarcyDev dv = D;
    void *kernels[3] = {reinterpret_cast<void *>(&k_darcy_matvec),
                        reinterpret_cast<void *>(&k_darcy_update),
                        reinterpret_cast<void *>(&k_darcy_direction)};
    for (int b = 0; b < len && e == hipSuccess; ++b) {
        int par = (par0 + b) & 1;
        void *args1[] = {&dv};
        void *args2[] = {&dv, &par};
        for (int k = 0; k < 3 && e == hipSuccess; ++k) {
            hipKernelNodeParams np;
            memset(&np, 0, sizeof(np));
            np.blockDim = dim3(kD);
            np.gridDim = dim3(D.nblk);
            np.func = kernels[k];
            np.kernelParams = k == 0 ? args1 : args2;
            hipGraphNode_t node = nullptr;
            e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &np);
            prev = node;
        }
    }
    if (e == hipSuccess) e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        set_error(std::string("Darcy iteration graph: ") + hipGetErrorString(e));
        return PAM_ERR_HIP;
    }
    return PAM_OK;
}

static pam_status darcy_setup(pam_ctx *ctx, const pam_darcy_opts *o, const double *k_tri,
                              double *p, DarcyDev &D) {
    const int n0 = o->n[0], n1 = o->n[1];
    const int64_t N = (int64_t)(n0 + 1) * (n1 + 1);
    const int nblk = (int)((N + kD - 1) / kD);
    size_t w = 0;
    auto take = [&](size_t bytes) { size_t r = w; w += (bytes + 255) / 256 * 256; return r; };
    const size_t o_wh = take(sizeof(double) * (size_t)(n1 + 1) * n0);
    const size_t o_wv = take(sizeof(double) * (size_t)n1 * (n0 + 1));
    const size_t o_vec = take(sizeof(double) * (size_t)N * 5);
    const size_t o_part = take(sizeof(double) * (size_t)nblk * 3);
    const size_t o_sc = take(sizeof(double) * 4);
    pam_status st = ensure(ctx, BUF_EVAL, w);
    if (st != PAM_OK) return st;
    char *b = wsp<char>(ctx, BUF_EVAL);
    D.n0 = n0;
    D.n1 = n1;
    const double hx = (o->hi[0] - o->lo[0]) / n0, hy = (o->hi[1] - o->lo[1]) / n1;
    D.cx = hy / (2.0 * hx);
    D.cy = hx / (2.0 * hy);
    D.p_left = o->p_left;
    D.p_right = o->p_right;
    D.k = k_tri;
    D.wh = (double *)(b + o_wh);
    D.wv = (double *)(b + o_wv);
    double *vec = (double *)(b + o_vec);
    D.diag = vec;
    D.r = vec + N;
    D.z = vec + 2 * N;
    D.d = vec + 3 * N;
    D.q = vec + 4 * N;
    D.x = p;
    D.part = (double *)(b + o_part);
    D.sc = (double *)(b + o_sc);
    D.nblk = nblk;
    return PAM_OK;
}

pam_status launch_darcy_solve(pam_ctx *ctx, const pam_darcy_opts *o, const double *k_tri,
                              double *p, int warm, int32_t *iters, double *rel_res) {
    DarcyDev D;
    pam_status st = darcy_setup(ctx, o, k_tri, p, D);
    if (st != PAM_OK) return st;
    const int ne = (D.n1 + 1) * D.n0 + D.n1 * (D.n0 + 1);
    KernelTimer kt(ctx, PAM_TK_DARCY);
    hipLaunchKernelGGL(k_darcy_edges, dim3((ne + kD - 1) / kD), dim3(kD), 0, ctx->stream, D);
    PAM_CHECK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_darcy_start, dim3(D.nblk), dim3(kD), 0, ctx->stream, D, warm);
    PAM_CHECK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_darcy_res, dim3(D.nblk), dim3(kD), 0, ctx->stream, D);
    PAM_CHECK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_darcy_init_scalars, dim3(1), dim3(kD), 0, ctx->stream, D);
    PAM_CHECK_HIP(hipGetLastError());
    double host_sc[4] = {0, 0, 0, 0};
    PAM_CHECK_HIP(hipMemcpyAsync(host_sc, D.sc, sizeof(host_sc), hipMemcpyDeviceToHost, ctx->stream));
    PAM_CHECK_HIP(hipStreamSynchronize(ctx->stream));
    const double bb = host_sc[3];
    int it = 0;
    double rel = bb > 0.0 ? sqrt(host_sc[2] / bb) : 0.0;
    hipGraphExec_t burst[2] = {nullptr, nullptr};   // by the parity of a burst's first iteration
    pam_status gst = PAM_OK;
    while (rel > o->tol && it < o->max_iter) {
        const int len = std::min(o->check_every, o->max_iter - it);
        if (len == o->check_every) {
            hipGraphExec_t &ex = burst[it & 1];
            if (!ex && (gst = build_burst(D, len, it & 1, &ex)) != PAM_OK) break;
            if (hipGraphLaunch(ex, ctx->stream) != hipSuccess) {
                set_error("hipGraphLaunch of the Darcy iteration failed");
                gst = PAM_ERR_HIP;
                break;
            }
            it += len;
        } else {   // a last, shorter burst
            for (int b = 0; b < len; ++b, ++it) {
                const int par = it & 1;
                hipLaunchKernelGGL(k_darcy_matvec, dim3(D.nblk), dim3(kD), 0, ctx->stream, D);
                hipLaunchKernelGGL(k_darcy_update, dim3(D.nblk), dim3(kD), 0, ctx->stream, D, par);
                hipLaunchKernelGGL(k_darcy_direction, dim3(D.nblk), dim3(kD), 0, ctx->stream, D, par);
            }
        }
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(host_sc, D.sc, sizeof(host_sc), hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
            hipStreamSynchronize(ctx->stream) != hipSuccess) {
            set_error("Darcy iteration failed");
            gst = PAM_ERR_HIP;
            break;
        }
        rel = bb > 0.0 ? sqrt(host_sc[2] / bb) : 0.0;
    }
    for (hipGraphExec_t ex : burst)
        if (ex) (void)hipGraphExecDestroy(ex);
    if (gst != PAM_OK) return gst;
    *iters = it;
    *rel_res = rel;
    return PAM_OK;
}

pam_status launch_darcy_error(pam_ctx *ctx, const pam_darcy_opts *o, const double *p_ref,
                              const double *p, double *e_rel) {
    const int n0 = o->n[0], n1 = o->n[1];
    const int ntri = 2 * n0 * n1;
    const int nblk = (ntri + kD - 1) / kD;
    size_t w = (sizeof(double) * 2 * nblk + 255) / 256 * 256 + 256;
    pam_status st = ensure(ctx, BUF_EVAL, w);
    if (st != PAM_OK) return st;
    double *part = wsp<double>(ctx, BUF_EVAL);
    double *out = part + 2 * nblk;
    const double area = (o->hi[0] - o->lo[0]) / n0 * (o->hi[1] - o->lo[1]) / n1 / 2.0;
    hipLaunchKernelGGL(k_darcy_norms, dim3(nblk), dim3(kD), 0, ctx->stream, n0, n1, area, p_ref, p,
                       part, nblk);
    PAM_CHECK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_darcy_norms_total, dim3(1), dim3(kD), 0, ctx->stream, part, nblk, out);
    PAM_CHECK_HIP(hipGetLastError());
    double h[2];
    PAM_CHECK_HIP(hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    PAM_CHECK_HIP(hipStreamSynchronize(ctx->stream));
    *e_rel = h[1] > 0.0 ? sqrt(h[0] / h[1]) : 0.0;
    return PAM_OK;
}

// ---------------------------------------------------------------- coefficient
// Centroids of the two triangles of every square of the mesh, [n1][n0][2][2]:
// lower-right (i,j),(i+1,j),(i+1,j+1) at ((x_i + 2 x_{i+1}) / 3, (2 y_j + y_{j+1}) / 3),
// upper-left (i,j),(i+1,j+1),(i,j+1) at ((2 x_i + x_{i+1}) / 3, (y_j + 2 y_{j+1}) / 3),
// with x_i = lo_0 + (hi_0 - lo_0) i / n0 and y_j likewise.
__global__ void __launch_bounds__(kD)
k_darcy_centroids(int n0, int n1, double lo0, double w0, double lo1, double w1,
                  double *__restrict__ xq) {
    const int64_t t = (int64_t)blockIdx.x * kD + threadIdx.x;
    if (t >= (int64_t)n0 * n1) return;
    const int i = (int)(t % n0), j = (int)(t / n0);
    const double x0 = lo0 + w0 * i / n0, x1 = lo0 + w0 * (i + 1) / n0;
    const double y0 = lo1 + w1 * j / n1, y1 = lo1 + w1 * (j + 1) / n1;
    double *q = xq + t * 4;
    q[0] = (x0 + 2.0 * x1) / 3.0;
    q[1] = (2.0 * y0 + y1) / 3.0;
    q[2] = (2.0 * x0 + x1) / 3.0;
    q[3] = (y0 + 2.0 * y1) / 3.0;
}

// The data's own coefficient: both triangles of square (i, j) take 10^y of
// data cell (i, j).
__global__ void __launch_bounds__(kD)
k_darcy_cells(int n0, int n1, const double *__restrict__ cell_y, double *__restrict__ k) {
    const int64_t t = (int64_t)blockIdx.x * kD + threadIdx.x;
    if (t >= (int64_t)n0 * n1) return;
    const double v = exp10(cell_y[t]);
    k[2 * t] = v;
    k[2 * t + 1] = v;
}

pam_status launch_darcy_coefficient(pam_ctx *ctx, const pam_darcy_opts *o, const pam_field *field,
                                    const pam_dict *dict, const double *beta, double blend,
                                    double *k_tri) {
    const int64_t nsq = (int64_t)o->n[0] * o->n[1];
    pam_status st = ensure(ctx, BUF_AUX, (size_t)nsq * 4 * sizeof(double));
    if (st != PAM_OK) return st;
    double *xq = wsp<double>(ctx, BUF_AUX);
    hipLaunchKernelGGL(k_darcy_centroids, dim3((unsigned)((nsq + kD - 1) / kD)), dim3(kD), 0,
                       ctx->stream, o->n[0], o->n[1], o->lo[0], o->hi[0] - o->lo[0], o->lo[1],
                       o->hi[1] - o->lo[1], xq);
    PAM_CHECK_HIP(hipGetLastError());
    pam_field f = *field;
    f.q_begin = 0;
    f.q_end = 2 * nsq;
    if (blend < 0.0)
        return launch_eval(ctx, 1, &f, dict, beta, 1, xq, 2 * nsq, k_tri, 1, nullptr);
    return launch_eval_blend(ctx, 1, &f, dict, beta, blend, 1, xq, 2 * nsq, k_tri, 1, nullptr);
}

pam_status launch_darcy_cells(pam_ctx *ctx, const pam_darcy_opts *o, const double *cell_y,
                              double *k_tri) {
    const int64_t nsq = (int64_t)o->n[0] * o->n[1];
    hipLaunchKernelGGL(k_darcy_cells, dim3((unsigned)((nsq + kD - 1) / kD)), dim3(kD), 0,
                       ctx->stream, o->n[0], o->n[1], cell_y, k_tri);
    PAM_CHECK_HIP(hipGetLastError());
    return PAM_OK;
}

}  // namespace pam
