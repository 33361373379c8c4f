// Partition/sample gathering and initial lattice dictionary (gfx950).
// Sec. 2 Step 1 (half-open box subdomains), Step 2 (one sample per element
// at its centroid, data vector of cell values); Exp. 1 (g x g lattice).
#include "pam_internal.h"

namespace pam {

struct GatherTable {
    int32_t first[3], last[3];  // cell-index range of the fit set per axis
};

// One block per (subdomain, 256 samples). Centroids lo + (i + 1/2) h use
// separately rounded multiply and add (contraction is off in these kernels,
// and the operations are written out rather than taken from header helpers
// whose arithmetic may still be fused after inlining), so that every consumer
// of the sample points sees identical bits.
__global__ void __launch_bounds__(256)
k_gather(int dim, int nc0, int nc1, double lo0, double lo1, double lo2, double h0, double h1,
         double h2, const GatherTable *__restrict__ tab, const int64_t *__restrict__ off,
         const double *__restrict__ cell_y, double *__restrict__ x, double *__restrict__ y,
         double *__restrict__ h, int32_t *__restrict__ cell) {
#pragma clang fp contract(off)
    const int s = blockIdx.y;
    const int64_t j0 = off[s];
    const int64_t N = off[s + 1] - j0;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= N) return;
    const GatherTable t = tab[s];
    const int64_t n0 = t.last[0] - t.first[0];
    const int64_t n1 = dim > 1 ? t.last[1] - t.first[1] : 1;
    int ii[3];
    ii[0] = t.first[0] + (int)(j % n0);
    ii[1] = dim > 1 ? t.first[1] + (int)((j / n0) % n1) : 0;
    ii[2] = dim > 2 ? t.first[2] + (int)(j / (n0 * n1)) : 0;
    const double lo[3] = {lo0, lo1, lo2};
    const double hh[3] = {h0, h1, h2};
    const int64_t g = (int64_t)ii[0] + (int64_t)nc0 * ((int64_t)ii[1] + (int64_t)nc1 * (int64_t)ii[2]);
    for (int a = 0; a < dim; ++a) {
        const double step = ((double)ii[a] + 0.5) * hh[a];  // rounded once
        x[(j0 + j) * dim + a] = lo[a] + step;            // rounded once
        h[(j0 + j) * dim + a] = hh[a];
        cell[(j0 + j) * dim + a] = ii[a];
    }
    y[j0 + j] = cell_y[g];
}

pam_status launch_gather(pam_ctx *ctx, const pam_grid *g, const void *tab_dev, int n_sub,
                         int32_t n_max, const double *cell_y, const int64_t *off, double *x,
                         double *y, double *h, int32_t *cell) {
    double hh[3] = {1.0, 1.0, 1.0};
    for (int a = 0; a < g->dim; ++a) hh[a] = (g->hi[a] - g->lo[a]) / (double)g->n_cells[a];
    dim3 grid((n_max + 255) / 256, n_sub);
    if (n_max <= 0) return PAM_OK;
    hipLaunchKernelGGL(k_gather, grid, dim3(256), 0, ctx->stream, g->dim, g->n_cells[0],
                       g->n_cells[1], g->lo[0], g->lo[1], g->lo[2], hh[0], hh[1], hh[2],
                       (const GatherTable *)tab_dev, off, cell_y, x, y, h, cell);
    PAM_CHECK_HIP(hipGetLastError());
    return PAM_OK;
}

struct LatticeTable {
    double lo[3], hc[3];  // owned box origin and lattice spacing per axis
    double sigma0;
};

// One block per subdomain: centers lo + (j + 1/2) h_c in row-major order
// (axis 0 fastest), widths sigma0, level 0.
__global__ void __launch_bounds__(256)
k_lattice(int dim, int g0, int g1, int g2, int m_cap, const LatticeTable *__restrict__ tab,
          int32_t *__restrict__ m, double *__restrict__ c, double *__restrict__ sigma,
          int32_t *__restrict__ level) {
#pragma clang fp contract(off)
    const int s = blockIdx.x;
    const int M = g0 * g1 * g2;
    const LatticeTable t = tab[s];
    for (int k = threadIdx.x; k < M; k += blockDim.x) {
        const int jj[3] = {k % g0, (k / g0) % g1, k / (g0 * g1)};
        for (int a = 0; a < dim; ++a)
            {
            const double step = ((double)jj[a] + 0.5) * t.hc[a];
            c[((size_t)s * m_cap + k) * dim + a] = t.lo[a] + step;
        }
        sigma[(size_t)s * m_cap + k] = t.sigma0;
        level[(size_t)s * m_cap + k] = 0;
    }
    if (threadIdx.x == 0) m[s] = M;
}

pam_status launch_lattice(pam_ctx *ctx, int dim, const int32_t *g, int n_sub, int m_cap,
                          const void *tab_dev, pam_dict *dict) {
    int gg[3] = {1, 1, 1};
    for (int a = 0; a < dim; ++a) gg[a] = g[a];
    hipLaunchKernelGGL(k_lattice, dim3(n_sub), dim3(256), 0, ctx->stream, dim, gg[0], gg[1], gg[2],
                       m_cap, (const LatticeTable *)tab_dev, dict->m, dict->c, dict->sigma,
                       dict->level);
    PAM_CHECK_HIP(hipGetLastError());
    return PAM_OK;
}

size_t gather_table_bytes(int n_sub) { return sizeof(GatherTable) * (size_t)n_sub; }
size_t lattice_table_bytes(int n_sub) { return sizeof(LatticeTable) * (size_t)n_sub; }

// Host-side construction of the launch tables (shared by count and gather).
// Fit range per axis: cells whose centroid index i + 1/2 lies in the owned
// interval [b_k, b_{k+1}) widened by overlap * width on interior faces.
void axis_range(int n_cells, int n_sub, const int32_t *brk, int k, double overlap, int *first,
                int *last) {
    const double b0 = (double)brk[k], b1 = (double)brk[k + 1];
    const double w = b1 - b0;
    double lo = b0, hi = b1;
    if (k > 0) lo = b0 - overlap * w;
    if (k < n_sub - 1) hi = b1 + overlap * w;
    int f = -1, l = -1;
    for (int i = 0; i < n_cells; ++i) {
        const double u = (double)i + 0.5;
        if (u >= lo && u < hi) {
            if (f < 0) f = i;
            l = i + 1;
        }
    }
    if (f < 0) f = l = 0;
    *first = f;
    *last = l;
}

void build_gather_table(const pam_grid *g, void *host_tab) {
    GatherTable *t = (GatherTable *)host_tab;
    const int32_t *brk[3] = {nullptr, nullptr, nullptr};
    int pos = 0;
    int ns[3] = {1, 1, 1};
    for (int a = 0; a < g->dim; ++a) {
        ns[a] = g->n_sub[a];
        brk[a] = g->breaks + pos;
        pos += g->n_sub[a] + 1;
    }
    int s = 0;
    for (int k2 = 0; k2 < ns[2]; ++k2)
        for (int k1 = 0; k1 < ns[1]; ++k1)
            for (int k0 = 0; k0 < ns[0]; ++k0, ++s) {
                const int kk[3] = {k0, k1, k2};
                for (int a = 0; a < 3; ++a) {
                    t[s].first[a] = 0;
                    t[s].last[a] = 1;
                }
                for (int a = 0; a < g->dim; ++a)
                    axis_range(g->n_cells[a], g->n_sub[a], brk[a], kk[a], g->overlap,
                               &t[s].first[a], &t[s].last[a]);
            }
}

void build_lattice_table(const pam_grid *g, const int32_t *gl, double sigma_factor, void *host_tab) {
    LatticeTable *t = (LatticeTable *)host_tab;
    const int32_t *brk[3] = {nullptr, nullptr, nullptr};
    int pos = 0;
    int ns[3] = {1, 1, 1};
    double hcell[3] = {1, 1, 1};
    for (int a = 0; a < g->dim; ++a) {
        ns[a] = g->n_sub[a];
        brk[a] = g->breaks + pos;
        pos += g->n_sub[a] + 1;
        hcell[a] = (g->hi[a] - g->lo[a]) / (double)g->n_cells[a];
    }
    int s = 0;
    for (int k2 = 0; k2 < ns[2]; ++k2)
        for (int k1 = 0; k1 < ns[1]; ++k1)
            for (int k0 = 0; k0 < ns[0]; ++k0, ++s) {
                const int kk[3] = {k0, k1, k2};
                double hmax = 0.0;
                for (int a = 0; a < 3; ++a) { t[s].lo[a] = 0.0; t[s].hc[a] = 0.0; }
                for (int a = 0; a < g->dim; ++a) {
                    volatile double blo = g->lo[a] + (double)brk[a][kk[a]] * hcell[a];
                    volatile double bhi = g->lo[a] + (double)brk[a][kk[a] + 1] * hcell[a];
                    t[s].lo[a] = blo;
                    t[s].hc[a] = (bhi - blo) / (double)gl[a];
                    if (t[s].hc[a] > hmax) hmax = t[s].hc[a];
                }
                t[s].sigma0 = sigma_factor * hmax;
            }
}

}  // namespace pam

namespace pam {

// Small fill and copy kernels: used instead of memset and device-to-device
// copy nodes wherever the work may be captured into a HIP graph.
__global__ void __launch_bounds__(256) k_fill_u32(uint32_t *__restrict__ p, uint32_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = v;
}

__global__ void __launch_bounds__(256) k_copy_i32(int32_t *__restrict__ d, const int32_t *__restrict__ s, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) d[i] = s[i];
}

pam_status launch_fill_u32(pam_ctx *ctx, void *p, uint32_t v, int64_t n) {
    if (n <= 0) return PAM_OK;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, ctx->stream, (uint32_t *)p, v, n);
    PAM_CHECK_HIP(hipGetLastError());
    return PAM_OK;
}

pam_status launch_copy_i32(pam_ctx *ctx, int32_t *d, const int32_t *s, int64_t n) {
    if (n <= 0) return PAM_OK;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_copy_i32, dim3(blocks), dim3(256), 0, ctx->stream, d, s, n);
    PAM_CHECK_HIP(hipGetLastError());
    return PAM_OK;
}

}  // namespace pam
