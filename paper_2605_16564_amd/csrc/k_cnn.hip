// Learned warm start for the elastic-net fits (gfx950): a four-layer 5x5
// "same" convolutional network on 16x16 cell patches of a subdomain
// (1 -> 32 -> 32 -> 32 -> 2 channels, ReLU after the first three layers).
// Output channel 0 is the refinement logit of each cell, channel 1 the logit
// that a center lying in the cell ends up active. The support channel seeds
// the starting active set of the exact solve (pam_enet_opts.support_hint);
// the solve's KKT certificate keeps its result the unique minimizer, so the
// network changes the work done, never the answer.
//
// Layout: activations FP32, channels first [B][C][16*16]; parameters FP32,
// per layer w[co][ci][5][5] then b[co], layers in order. A pack kernel
// re-lays the weights per call into the forward order [ci][tap][co] and the
// backward-data order (flipped taps, in/out swapped), so that the output
// channel weights a thread needs at one (ci, tap) are contiguous and
// wave-uniform (scalar loads).
//
// Kernels: direct convolution with the padded input plane in LDS and one
// output pixel per thread (forward, and backward-data as a forward pass over
// the packed flipped weights, with the ReLU gate fused); weight gradients as
// per-block partial sums with a 5x5 register window sliding along each row;
// masked BCE-with-logits; Adam; patch extraction and the hint map.
#include <float.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "pam_internal.h"

namespace pam {

static constexpr int kP = 16;           // patch side
static constexpr int kPix = kP * kP;    // pixels per patch (one thread each)
static constexpr int kK = 5;            // kernel side
static constexpr int kTaps = kK * kK;
static constexpr int kH = kP + kK - 1;  // padded side
static constexpr int kHs = kH + 1;      // padded LDS row stride (bank spread)
static constexpr int kGs = kPix + 1;    // LDS row stride of gradient planes

__host__ __device__ constexpr int cnn_cin(int l) { return l == 0 ? 1 : 32; }
__host__ __device__ constexpr int cnn_cout(int l) { return l == 3 ? 2 : 32; }
__host__ __device__ constexpr int layer_size(int l) {
    return cnn_cout(l) * cnn_cin(l) * kTaps + cnn_cout(l);
}
__host__ __device__ constexpr int cnn_off(int l) {
    return l == 0 ? 0 : cnn_off(l - 1) + layer_size(l - 1);
}
static constexpr int kParams = cnn_off(4);
static_assert(kParams == 53698, "parameter count of the 1-32-32-32-2 network");

// ---------------------------------------------------------------- packing
// wf: [ci][tap][co] (forward), wb: [co][tap'][ci] with tap' the point-
// reflected tap (backward data, a forward pass from cout to cin channels);
// both at the layer's parameter offset, biases untouched.
__global__ void k_pack(const float *__restrict__ params, float *__restrict__ wf, float *__restrict__ wb) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kParams) return;
    int l = 0;
    while (l < 3 && e >= cnn_off(l + 1)) ++l;
    const int r = e - cnn_off(l), ci_n = cnn_cin(l), co_n = cnn_cout(l);
    if (r >= co_n * ci_n * kTaps) return;   // bias
    const int co = r / (ci_n * kTaps), ci = (r / kTaps) % ci_n, tap = r % kTaps;
    const float w = params[e];
    wf[cnn_off(l) + (ci * kTaps + tap) * co_n + co] = w;
    wb[cnn_off(l) + (co * kTaps + (kTaps - 1 - tap)) * ci_n + ci] = w;
}

// ---------------------------------------------------------------- conv
// out[b][co][p] = bias[co] + sum_ci sum_tap w[ci][tap][co] in[b][ci][p + tap - 2]
// mode 0: identity, 1: ReLU, 2: gate (out = gate > 0 ? v : 0)
template <int CIN, int COUT>
__global__ void __launch_bounds__(kPix)
k_conv(const float *__restrict__ in, const float *__restrict__ w, const float *__restrict__ bias,
       float *__restrict__ out, int mode, const float *__restrict__ gate) {
    __shared__ float sx[CIN][kH][kHs];
    const int b = blockIdx.x;
    const int py = threadIdx.x / kP, px = threadIdx.x % kP;
    const float *src = in + (size_t)b * CIN * kPix;
    for (int e = threadIdx.x; e < CIN * kH * kH; e += kPix) {
        const int ci = e / (kH * kH), r = e % (kH * kH);
        const int yy = r / kH - 2, xx = r % kH - 2;
        sx[ci][r / kH][r % kH] = (yy >= 0 && yy < kP && xx >= 0 && xx < kP) ? src[ci * kPix + yy * kP + xx] : 0.0f;
    }
    __syncthreads();
    float acc[COUT];
#pragma unroll
    for (int co = 0; co < COUT; ++co) acc[co] = bias ? bias[co] : 0.0f;
    for (int ci = 0; ci < CIN; ++ci) {
        const float *wc = w + ci * kTaps * COUT;
#pragma unroll 1
        for (int ky = 0; ky < kK; ++ky)
#pragma unroll
            for (int kx = 0; kx < kK; ++kx) {
                const float xv = sx[ci][py + ky][px + kx];
                const float *wt = wc + (ky * kK + kx) * COUT;
#pragma unroll
                for (int co = 0; co < COUT; ++co) acc[co] += wt[co] * xv;
            }
    }
    float *dst = out + (size_t)b * COUT * kPix + threadIdx.x;
    const float *gt = gate ? gate + (size_t)b * COUT * kPix + threadIdx.x : nullptr;
#pragma unroll
    for (int co = 0; co < COUT; ++co) {
        float v = acc[co];
        if (mode == 1) v = fmaxf(v, 0.0f);
        else if (mode == 2) v = gt[co * kPix] > 0.0f ? v : 0.0f;
        dst[co * kPix] = v;
    }
}

// Weight (and bias) gradient partial sums of one block over patches
// [b0, b1): thread = (ci, group of CG output channels, row group g); it
// keeps CG x 25 accumulators and slides a 5x5 input window along each row.
// part[(blk * G + g)][co*CIN*25 + ci*25 + tap], bias at [COUT*CIN*25 + co].
template <int CIN, int COUT, int CG, int G>
__global__ void __launch_bounds__(CIN * (COUT / CG) * G)
k_wgrad(const float *__restrict__ in, const float *__restrict__ gout, int B, int per_block,
        float *__restrict__ part) {
    constexpr int NG = COUT / CG, NT = CIN * NG, NTH = NT * G;
    constexpr int NW = COUT * CIN * kTaps + COUT;
    __shared__ float sx[CIN][kH][kHs];
    __shared__ float sg[COUT][kGs];
    const int t = threadIdx.x, pair = t % NT, g = t / NT;
    const int ci = pair / NG, co0 = (pair % NG) * CG;
    float acc[CG][kTaps], accb[CG];
#pragma unroll
    for (int c = 0; c < CG; ++c) {
        accb[c] = 0.0f;
#pragma unroll
        for (int k = 0; k < kTaps; ++k) acc[c][k] = 0.0f;
    }
    const int b0 = blockIdx.x * per_block, b1 = min(B, b0 + per_block);
    for (int b = b0; b < b1; ++b) {
        const float *src = in + (size_t)b * CIN * kPix;
        for (int e = t; e < CIN * kH * kH; e += NTH) {
            const int cc = e / (kH * kH), r = e % (kH * kH);
            const int yy = r / kH - 2, xx = r % kH - 2;
            sx[cc][r / kH][r % kH] =
                (yy >= 0 && yy < kP && xx >= 0 && xx < kP) ? src[cc * kPix + yy * kP + xx] : 0.0f;
        }
        const float *gsrc = gout + (size_t)b * COUT * kPix;
        for (int e = t; e < COUT * kPix; e += NTH) sg[e / kPix][e % kPix] = gsrc[e];
        __syncthreads();
        for (int py = g; py < kP; py += G) {
            float win[kK][kK];
#pragma unroll
            for (int ky = 0; ky < kK; ++ky)
#pragma unroll
                for (int kx = 0; kx < kK - 1; ++kx) win[ky][kx + 1] = sx[ci][py + ky][kx];
            for (int px = 0; px < kP; ++px) {
#pragma unroll
                for (int ky = 0; ky < kK; ++ky) {
#pragma unroll
                    for (int kx = 0; kx < kK - 1; ++kx) win[ky][kx] = win[ky][kx + 1];
                    win[ky][kK - 1] = sx[ci][py + ky][px + kK - 1];
                }
#pragma unroll
                for (int c = 0; c < CG; ++c) {
                    const float gv = sg[co0 + c][py * kP + px];
                    accb[c] += gv;
#pragma unroll
                    for (int ky = 0; ky < kK; ++ky)
#pragma unroll
                        for (int kx = 0; kx < kK; ++kx) acc[c][ky * kK + kx] += gv * win[ky][kx];
                }
            }
        }
        __syncthreads();
    }
    float *dst = part + ((size_t)blockIdx.x * G + g) * NW;
#pragma unroll
    for (int c = 0; c < CG; ++c) {
#pragma unroll
        for (int k = 0; k < kTaps; ++k) dst[((co0 + c) * CIN + ci) * kTaps + k] = acc[c][k];
        if (ci == 0) dst[COUT * CIN * kTaps + co0 + c] = accb[c];
    }
}

// sum of n_part partial gradient rows into the layer's gradient slice:
// 64 outputs per block, four slices of the partial rows per output (eight
// rows in flight per thread), combined in LDS in a fixed order.
__global__ void __launch_bounds__(256)
k_wgrad_reduce(const float *__restrict__ part, int n_part, int nw, float *__restrict__ grad) {
    const int o = blockIdx.x * 64 + (threadIdx.x & 63), sl = threadIdx.x >> 6;
    float acc = 0.0f;
    if (o < nw) {
        int p = sl;
        for (; p + 28 < n_part; p += 32) {
            float v[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = part[(size_t)(p + 4 * e) * nw + o];
#pragma unroll
            for (int e = 0; e < 8; ++e) acc += v[e];
        }
        for (; p < n_part; p += 4) acc += part[(size_t)p * nw + o];
    }
    __shared__ float red[4][64];
    red[sl][threadIdx.x & 63] = acc;
    __syncthreads();
    if (sl == 0 && o < nw) grad[o] = (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

// ---------------------------------------------------------------- loss
// masked binary cross-entropy with logits over n entries:
// loss = sum mask * (max(z,0) - z t + log(1 + exp(-|z|))) / sum mask and
// d loss / d z = mask (sigmoid(z) - t) / sum mask. Pass 1 writes the
// unscaled gradient and per-block partial sums; pass 2 scales.
static constexpr int kBceBlocks = 512;

__global__ void __launch_bounds__(256)
k_bce(const float *__restrict__ z, const float *__restrict__ tg, const float *__restrict__ mk,
      int64_t n, float *__restrict__ grad, float *__restrict__ part) {
    float l = 0.0f, c = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const float zz = z[i], tt = tg[i], mm = mk[i];
        const float e = expf(-fabsf(zz));
        const float sig = zz >= 0.0f ? 1.0f / (1.0f + e) : e / (1.0f + e);
        l += mm * (fmaxf(zz, 0.0f) - zz * tt + log1pf(e));
        c += mm;
        grad[i] = mm * (sig - tt);
    }
    __shared__ float rl[4], rc[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        l += __shfl_xor(l, o, 64);
        c += __shfl_xor(c, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        rl[threadIdx.x >> 6] = l;
        rc[threadIdx.x >> 6] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = rl[0] + rl[1] + rl[2] + rl[3];
        part[2 * blockIdx.x + 1] = rc[0] + rc[1] + rc[2] + rc[3];
    }
}

__global__ void __launch_bounds__(256)
k_bce_scale(const float *__restrict__ part, int nb, float *__restrict__ grad, int64_t n,
            float *__restrict__ loss) {
    __shared__ double tl[256], tc[256];
    double l = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) {
        l += part[2 * i];
        c += part[2 * i + 1];
    }
    tl[threadIdx.x] = l;
    tc[threadIdx.x] = c;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            tl[threadIdx.x] += tl[threadIdx.x + s];
            tc[threadIdx.x] += tc[threadIdx.x + s];
        }
        __syncthreads();
    }
    const double cnt = tc[0];
    const float inv = cnt > 0.0 ? (float)(1.0 / cnt) : 0.0f;
    if (blockIdx.x == 0 && threadIdx.x == 0 && loss) *loss = cnt > 0.0 ? (float)(tl[0] / cnt) : 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        grad[i] *= inv;
}

__global__ void k_fill(float *__restrict__ p, int64_t n, float v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Adam (Kingma and Ba 2015) with bias correction; c1 = 1 - beta1^t, c2 = 1 - beta2^t
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------- patches
// Subdomain s owns cells [i0, i0+ni) x [j0, j0+nj) (multiples of 16); its
// patches are numbered row-major over the patch grid from pbase[s]; value =
// scale * y of the cell.
__global__ void __launch_bounds__(kPix)
k_patches(int nc0, const int32_t *__restrict__ box, const int32_t *__restrict__ pbase,
          const double *__restrict__ cell_y, float scale, float *__restrict__ patches) {
    const int s = blockIdx.y, pl = blockIdx.x;
    const int i0 = box[4 * s], j0 = box[4 * s + 1], ni = box[4 * s + 2] / kP, nj = box[4 * s + 3] / kP;
    if (pl >= ni * nj) return;
    const int pi = pl % ni, pj = pl / ni;
    const int x = i0 + pi * kP + threadIdx.x % kP, y = j0 + pj * kP + threadIdx.x / kP;
    patches[(size_t)(pbase[s] + pl) * kPix + threadIdx.x] = (float)(scale * cell_y[(size_t)y * nc0 + x]);
}

// Center k of subdomain s is hinted active when the support logit of the
// patch cell containing it (floor of the cell coordinate, clamped to the
// owned box) exceeds thr.
__global__ void __launch_bounds__(256)
k_hint(int m_cap, const int32_t *__restrict__ m, const double *__restrict__ c,
       const int32_t *__restrict__ box, const int32_t *__restrict__ pbase, double lo0, double lo1,
       double h0, double h1, const float *__restrict__ logits, float thr, uint8_t *__restrict__ hint) {
    const int s = blockIdx.y;
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= m_cap) return;
    uint8_t out = 0;
    const int M = max(0, min(m[s], m_cap));
    if (k < M) {
        const int i0 = box[4 * s], j0 = box[4 * s + 1], ni = box[4 * s + 2], nj = box[4 * s + 3];
        const double cx = c[((size_t)s * m_cap + k) * 2], cy = c[((size_t)s * m_cap + k) * 2 + 1];
        int ix = (int)floor((cx - lo0) / h0) - i0, iy = (int)floor((cy - lo1) / h1) - j0;
        ix = min(max(ix, 0), ni - 1);
        iy = min(max(iy, 0), nj - 1);
        const int pl = (iy / kP) * (ni / kP) + ix / kP;
        const int pix = (iy % kP) * kP + ix % kP;
        out = logits[((size_t)(pbase[s] + pl) * 2 + 1) * kPix + pix] > thr ? 1 : 0;
    }
    hint[(size_t)s * m_cap + k] = out;
}

// Training labels from the method's own results. Pass 1 (centers): the
// support channel of every cell holding a center gets mask 1, target 0;
// pass 2 sets target 1 where a center in the cell has beta != 0 (any active
// center marks its cell). Samples: the refinement channel of the owned cell
// of every sample gets mask 1 and target (elem_level > 0). Cells are found
// from coordinates by floor((x - lo) / h), as in the hint map.
__device__ __forceinline__ int patch_pixel(const int32_t *box, const int32_t *pbase, int s, int ix, int iy) {
    const int ni = box[4 * s + 2];
    return (pbase[s] + (iy / kP) * (ni / kP) + ix / kP) * 2 * kPix + (iy % kP) * kP + ix % kP;
}

__global__ void __launch_bounds__(256)
k_label_centers(int m_cap, const int32_t *__restrict__ m, const double *__restrict__ c,
                const double *__restrict__ beta, const int32_t *__restrict__ box,
                const int32_t *__restrict__ pbase, double lo0, double lo1, double h0, double h1, int pass,
                float *__restrict__ target, float *__restrict__ mask) {
    const int s = blockIdx.y, k = blockIdx.x * 256 + threadIdx.x;
    if (k >= max(0, min(m[s], m_cap))) return;
    const double cx = c[((size_t)s * m_cap + k) * 2], cy = c[((size_t)s * m_cap + k) * 2 + 1];
    int ix = (int)floor((cx - lo0) / h0) - box[4 * s], iy = (int)floor((cy - lo1) / h1) - box[4 * s + 1];
    ix = min(max(ix, 0), box[4 * s + 2] - 1);
    iy = min(max(iy, 0), box[4 * s + 3] - 1);
    const int at = patch_pixel(box, pbase, s, ix, iy) + kPix;   // support channel
    if (pass == 0) {
        mask[at] = 1.0f;
        target[at] = 0.0f;
    } else if (beta[(size_t)s * m_cap + k] != 0.0) {
        target[at] = 1.0f;
    }
}

__global__ void __launch_bounds__(256)
k_label_samples(const int64_t *__restrict__ off, const double *__restrict__ x,
                const int32_t *__restrict__ elem_level, const int32_t *__restrict__ box,
                const int32_t *__restrict__ pbase, double lo0, double lo1, double h0, double h1,
                float *__restrict__ target, float *__restrict__ mask) {
    const int s = blockIdx.y;
    const int64_t j = off[s] + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= off[s + 1]) return;
    const int ix = (int)floor((x[2 * j] - lo0) / h0) - box[4 * s];
    const int iy = (int)floor((x[2 * j + 1] - lo1) / h1) - box[4 * s + 1];
    if (ix < 0 || iy < 0 || ix >= box[4 * s + 2] || iy >= box[4 * s + 3]) return;   // overlap cells
    const int at = patch_pixel(box, pbase, s, ix, iy);
    mask[at] = 1.0f;
    target[at] = elem_level[j] > 0 ? 1.0f : 0.0f;
}

// ---------------------------------------------------------------- BF16 MFMA path
// The 32 -> 32 layers as implicit GEMMs on the matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation): operand A lane l holds row
// l % 16 and reduction elements 8 (l / 16) .. +7, operand B column l % 16 and
// the same reduction elements; D lane l holds rows 4 (l / 16) .. +3 of
// column l % 16.
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short to_bf16(float f) {
    // round to nearest even
    unsigned int u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

// BF16 weight packs of the 32 -> 32 layers l = 1, 2: forward [co][tap][ci]
// and backward-data [ci][tap'][co] (tap' the point-reflected tap).
__global__ void k_pack_bf16(const float *__restrict__ params, unsigned short *__restrict__ wf,
                            unsigned short *__restrict__ wb) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 2 * 32 * 32 * kTaps) return;
    const int l = 1 + e / (32 * 32 * kTaps), r = e % (32 * 32 * kTaps);
    const int co = r / (32 * kTaps), ci = (r / kTaps) % 32, tap = r % kTaps;
    const unsigned short w = to_bf16(params[cnn_off(l) + r]);
    unsigned short *f = wf + (size_t)(l - 1) * 32 * 32 * kTaps, *b = wb + (size_t)(l - 1) * 32 * 32 * kTaps;
    f[(co * kTaps + tap) * 32 + ci] = w;
    b[(ci * kTaps + (kTaps - 1 - tap)) * 32 + co] = w;
}

// out[b][o][p] = bias[o] + sum_tap sum_c w[o][tap][c] in[b][c][p + tap - 2]
// for 32 input and 32 output channels; mode 0 identity, 1 ReLU, 2 gate.
// 256 threads: wave w computes pixel rows 4w .. 4w+3 for both 16-channel
// output tiles. The padded input plane is staged channels-last in BF16.
static constexpr int kCs = 40;   // LDS channel stride (80 B: 16-byte aligned, spreads banks)

__global__ void __launch_bounds__(256)
k_conv32_mfma(const float *__restrict__ in, const unsigned short *__restrict__ w, const float *__restrict__ bias,
              float *__restrict__ out, int mode, const float *__restrict__ gate, int B) {
    __shared__ __attribute__((aligned(16))) unsigned short sx[kH][kH][kCs];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int col = lane & 15, kq = 8 * (lane >> 4);
    for (int b = blockIdx.x; b < B; b += gridDim.x) {
        __syncthreads();
        const float *src = in + (size_t)b * 32 * kPix;
        for (int e = threadIdx.x; e < 32 * kH * kH; e += 256) {
            const int c = e / (kH * kH), rr = e % (kH * kH);
            const int yy = rr / kH - 2, xx = rr % kH - 2;
            const float v = (yy >= 0 && yy < kP && xx >= 0 && xx < kP) ? src[c * kPix + yy * kP + xx] : 0.0f;
            sx[rr / kH][rr % kH][c] = to_bf16(v);
        }
        __syncthreads();
        v4f acc[4][2];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            acc[r][0] = v4f{0.f, 0.f, 0.f, 0.f};
            acc[r][1] = v4f{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll 1
        for (int tap = 0; tap < kTaps; ++tap) {
            const int ky = tap / kK, kx = tap % kK;
            const v8bf a0 = *reinterpret_cast<const v8bf *>(w + ((size_t)col * kTaps + tap) * 32 + kq);
            const v8bf a1 = *reinterpret_cast<const v8bf *>(w + ((size_t)(16 + col) * kTaps + tap) * 32 + kq);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int py = 4 * wv + r;
                const v8bf bv = *reinterpret_cast<const v8bf *>(&sx[py + ky][col + kx][kq]);
                acc[r][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bv, acc[r][0], 0, 0, 0);
                acc[r][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bv, acc[r][1], 0, 0, 0);
            }
        }
        float *dst = out + (size_t)b * 32 * kPix;
        const float *gt = gate ? gate + (size_t)b * 32 * kPix : nullptr;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int o = 16 * t + 4 * (lane >> 4) + q;
                    const int pp = (4 * wv + r) * kP + col;
                    float v = acc[r][t][q] + (bias ? bias[o] : 0.0f);
                    if (mode == 1) v = fmaxf(v, 0.0f);
                    else if (mode == 2) v = gt[o * kPix + pp] > 0.0f ? v : 0.0f;
                    dst[o * kPix + pp] = v;
                }
    }
}

// Weight and bias gradient partials of a 32 -> 32 layer over patches
// [b0, b1): gw[o][c][tap] = sum_p gout[o][p] in[c][p + tap - 2]. The
// reduction runs over pixels, 32 per MFMA (two rows); the input is staged as
// five column-shifted BF16 copies so that every 8-pixel fragment is aligned.
// Wave w owns the (tap, input-tile) pairs w, w+4, ... (50 pairs, two
// output tiles each). part[blk][o*800 + c*25 + tap], bias at [25600 + o].
__global__ void __launch_bounds__(256)
k_wgrad32_mfma(const float *__restrict__ in, const float *__restrict__ gout, int B, int per_block,
               float *__restrict__ part) {
    constexpr int NP = 13;   // pairs per wave (50 over 4 waves)
    __shared__ __attribute__((aligned(16))) unsigned short xs[kK][32][kH][kP];   // [kx][c][row][col]
    __shared__ __attribute__((aligned(16))) unsigned short gs[32][kPix];         // [o][p]
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int col = lane & 15, kq = 8 * (lane >> 4);
    v4f acc[NP][2];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        acc[i][0] = v4f{0.f, 0.f, 0.f, 0.f};
        acc[i][1] = v4f{0.f, 0.f, 0.f, 0.f};
    }
    float bacc = 0.0f;   // bias gradient: thread o < 32 sums gout[o][.]
    const int b0 = blockIdx.x * per_block, b1 = min(B, b0 + per_block);
    for (int b = b0; b < b1; ++b) {
        __syncthreads();
        const float *src = in + (size_t)b * 32 * kPix;
        // two adjacent columns per thread and 32-bit store
        for (int e = threadIdx.x; e < kK * 32 * kH * (kP / 2); e += 256) {
            const int kx = e / (32 * kH * (kP / 2)), r1 = e % (32 * kH * (kP / 2));
            const int c = r1 / (kH * (kP / 2)), r2 = r1 % (kH * (kP / 2));
            const int row = r2 / (kP / 2), cl = 2 * (r2 % (kP / 2));
            const int yy = row - 2, x0 = cl + kx - 2;
            const bool ry = yy >= 0 && yy < kP;
            const float v0 = (ry && x0 >= 0 && x0 < kP) ? src[c * kPix + yy * kP + x0] : 0.0f;
            const float v1 = (ry && x0 + 1 >= 0 && x0 + 1 < kP) ? src[c * kPix + yy * kP + x0 + 1] : 0.0f;
            *reinterpret_cast<unsigned int *>(&xs[kx][c][row][cl]) =
                (unsigned int)to_bf16(v0) | ((unsigned int)to_bf16(v1) << 16);
        }
        const float *g = gout + (size_t)b * 32 * kPix;
        for (int e = threadIdx.x; e < 32 * kPix / 2; e += 256) {
            const float2 gv = reinterpret_cast<const float2 *>(g)[e];
            reinterpret_cast<unsigned int *>(&gs[0][0])[e] = (unsigned int)to_bf16(gv.x) | ((unsigned int)to_bf16(gv.y) << 16);
        }
        {
            // bias: 8 threads per output channel, 32 pixels each
            const int o = threadIdx.x >> 3, sg = threadIdx.x & 7;
            float t = 0.0f;
            for (int p2 = 0; p2 < 32; ++p2) t += g[o * kPix + sg * 32 + p2];
            t += __shfl_xor(t, 1, 64);
            t += __shfl_xor(t, 2, 64);
            t += __shfl_xor(t, 4, 64);
            bacc += t;   // lanes with sg == 0 keep the channel's sum
        }
        __syncthreads();
        // 8 reduction chunks of 32 pixels (rows 2j, 2j+1)
        for (int j = 0; j < kP / 2; ++j) {
            // this lane's 8 pixels: row 2j + (kq >= 16), columns (kq % 16) .. +7
            const int prow = 2 * j + (kq >> 4), pcol = kq & 15;
            const v8bf a0 = *reinterpret_cast<const v8bf *>(&gs[col][prow * kP + pcol]);
            const v8bf a1 = *reinterpret_cast<const v8bf *>(&gs[16 + col][prow * kP + pcol]);
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                const int pr = wv + 4 * i;
                if (pr < 2 * kTaps) {
                    const int tap = pr >> 1, ct = pr & 1;
                    const int ky = tap / kK, kx = tap % kK;
                    const v8bf bv = *reinterpret_cast<const v8bf *>(&xs[kx][16 * ct + col][prow + ky][pcol]);
                    acc[i][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bv, acc[i][0], 0, 0, 0);
                    acc[i][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bv, acc[i][1], 0, 0, 0);
                }
            }
        }
    }
    float *dst = part + (size_t)blockIdx.x * (32 * 32 * kTaps + 32);
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const int pr = wv + 4 * i;
        if (pr >= 2 * kTaps) continue;
        const int tap = pr >> 1, ct = pr & 1;
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int o = 16 * t + 4 * (lane >> 4) + q, c = 16 * ct + col;
                dst[(o * 32 + c) * kTaps + tap] = acc[i][t][q];
            }
    }
    if ((threadIdx.x & 7) == 0) dst[32 * 32 * kTaps + (threadIdx.x >> 3)] = bacc;
}

// ---------------------------------------------------------------- launchers
struct CnnWs {
    float *wf, *wb, *a[3], *z, *ga, *gb, *gz, *part, *bpart;
    unsigned short *hf, *hb;   // BF16 packs of the 32 -> 32 layers (forward, backward data)
};
static constexpr int kPack16 = 2 * 32 * 32 * kTaps;   // BF16 elements per pack

static constexpr int kWgradPer = 8;     // patches per weight-gradient block (vector ALU kernels)
static constexpr int kWgradPerThin = 2; // the same for the thin first and last layers: their
                                        // blocks are small (128 / 256 threads), so more of them
static constexpr int kWgradPer16 = 4;   // patches per block of the MFMA weight gradient

static size_t cnn_ws_floats(int B, bool train) {
    const size_t A = (size_t)B * 32 * kPix;
    size_t n = 2 * (size_t)kParams + 3 * A + (size_t)B * 2 * kPix + kPack16;   // two BF16 packs = kPack16 floats
    if (train) {
        // partial gradient rows of the largest layer: thin layers 16 (first) or
        // 8 (last) rows per block, the 32 -> 32 layers one per block
        const size_t nblk = (B + kWgradPer - 1) / kWgradPer;
        const size_t nthin = (B + kWgradPerThin - 1) / kWgradPerThin;
        const size_t nblk16 = (B + kWgradPer16 - 1) / kWgradPer16;
        const size_t part = std::max({nthin * 16 * (size_t)layer_size(0), nthin * 8 * (size_t)layer_size(3),
                                      std::max(nblk, nblk16) * (size_t)layer_size(1)});
        n += 2 * A + (size_t)B * 2 * kPix + 2 * kBceBlocks + part;
    }
    return n;
}

static CnnWs carve(float *p, int B, bool train) {
    const size_t A = (size_t)B * 32 * kPix;
    CnnWs w{};
    w.wf = p; p += kParams;
    w.wb = p; p += kParams;
    for (int i = 0; i < 3; ++i) { w.a[i] = p; p += A; }
    w.z = p; p += (size_t)B * 2 * kPix;
    w.hf = reinterpret_cast<unsigned short *>(p);
    w.hb = w.hf + kPack16;
    p += kPack16;
    if (train) {
        w.ga = p; p += A;
        w.gb = p; p += A;
        w.gz = p; p += (size_t)B * 2 * kPix;
        w.bpart = p; p += 2 * kBceBlocks;
        w.part = p;
    }
    return w;
}

static void conv(pam_ctx *ctx, int cin, int cout, const float *in, const float *w, const float *b,
                 float *out, int B, int mode, const float *gate) {
    const dim3 g(B), t(kPix);
    if (cin == 1) hipLaunchKernelGGL((k_conv<1, 32>), g, t, 0, ctx->stream, in, w, b, out, mode, gate);
    else if (cout == 32 && cin == 32) hipLaunchKernelGGL((k_conv<32, 32>), g, t, 0, ctx->stream, in, w, b, out, mode, gate);
    else if (cout == 2) hipLaunchKernelGGL((k_conv<32, 2>), g, t, 0, ctx->stream, in, w, b, out, mode, gate);
    else hipLaunchKernelGGL((k_conv<2, 32>), g, t, 0, ctx->stream, in, w, b, out, mode, gate);
}

static int mfma_grid(int B) { return std::min(B, 4096); }

static void forward(pam_ctx *ctx, const float *params, const CnnWs &w, const float *x, float *z, int B, bool bf16) {
    hipLaunchKernelGGL(k_pack, dim3((kParams + 255) / 256), dim3(256), 0, ctx->stream, params, w.wf, w.wb);
    if (bf16)
        hipLaunchKernelGGL(k_pack_bf16, dim3((kPack16 + 255) / 256), dim3(256), 0, ctx->stream, params, w.hf, w.hb);
    const float *in = x;
    for (int l = 0; l < 4; ++l) {
        float *out = l < 3 ? w.a[l] : z;
        const float *bias = params + cnn_off(l) + cnn_cout(l) * cnn_cin(l) * kTaps;
        if (bf16 && (l == 1 || l == 2))
            hipLaunchKernelGGL(k_conv32_mfma, dim3(mfma_grid(B)), dim3(256), 0, ctx->stream, in,
                               w.hf + (size_t)(l - 1) * 32 * 32 * kTaps, bias, out, 1, (const float *)nullptr, B);
        else
            conv(ctx, cnn_cin(l), cnn_cout(l), in, w.wf + cnn_off(l), bias, out, B, l < 3 ? 1 : 0, nullptr);
        in = out;
    }
}

static pam_status check_prec(int precision) {
    PAM_REQUIRE(precision == PAM_PREC_F32 || precision == PAM_PREC_BF16,
                "network precision must be PAM_PREC_F32 or PAM_PREC_BF16");
    return PAM_OK;
}

static pam_status check_ctx(pam_ctx *ctx) {
    if (!ctx || !ctx->alive) {
        set_error("invalid context");
        return PAM_ERR_STATE;
    }
    return PAM_OK;
}

// Host table of the patch cut: per subdomain the owned cell box
// (i0, j0, ni, nj), then per subdomain the index of its first patch.
static pam_status patch_table(const pam_grid *g, std::vector<int32_t> &tab, int *n_patch, int *max_per) {
    PAM_REQUIRE(g && g->dim == 2 && g->breaks, "patches need a 2-D grid with breakpoints");
    const int n0 = g->n_sub[0], n1 = g->n_sub[1];
    PAM_REQUIRE(n0 >= 1 && n1 >= 1, "empty partition");
    const int32_t *b0 = g->breaks, *b1 = g->breaks + n0 + 1;
    const int n_sub = n0 * n1;
    tab.assign((size_t)5 * n_sub, 0);
    int tot = 0, mx = 0;
    for (int k1 = 0; k1 < n1; ++k1)
        for (int k0 = 0; k0 < n0; ++k0) {
            const int s = k0 + n0 * k1;
            const int ni = b0[k0 + 1] - b0[k0], nj = b1[k1 + 1] - b1[k1];
            PAM_REQUIRE(ni > 0 && nj > 0 && ni % kP == 0 && nj % kP == 0,
                        "owned boxes must be positive multiples of 16 cells per axis");
            tab[4 * s] = b0[k0];
            tab[4 * s + 1] = b1[k1];
            tab[4 * s + 2] = ni;
            tab[4 * s + 3] = nj;
            tab[4 * n_sub + s] = tot;
            tot += (ni / kP) * (nj / kP);
            mx = std::max(mx, (ni / kP) * (nj / kP));
        }
    *n_patch = tot;
    *max_per = mx;
    return PAM_OK;
}

}  // namespace pam

using namespace pam;

extern "C" {

int64_t pam_cnn_param_count(void) { return kParams; }

pam_status pam_cnn_forward(pam_ctx *ctx, const float *params, int32_t B, const float *x, float *logits,
                           int32_t precision) {
    pam_status st = check_ctx(ctx);
    if (st != PAM_OK) return st;
    if ((st = check_prec(precision)) != PAM_OK) return st;
    PAM_REQUIRE(params && x && logits && B >= 1, "NULL argument or B < 1");
    PAM_CHECK_HIP(hipSetDevice(ctx->device));
    if ((st = ensure(ctx, BUF_CNN, cnn_ws_floats(B, false) * sizeof(float))) != PAM_OK) return st;
    const CnnWs w = carve(wsp<float>(ctx, BUF_CNN), B, false);
    KernelTimer kt(ctx, PAM_TK_CNN);
    forward(ctx, params, w, x, logits, B, precision == PAM_PREC_BF16);
    PAM_CHECK_HIP(hipGetLastError());
    return PAM_OK;
}

pam_status pam_cnn_loss_grad(pam_ctx *ctx, const float *params, int32_t B, const float *x,
                             const float *target, const float *mask, float *grads, float *loss,
                             int32_t precision) {
    pam_status st = check_ctx(ctx);
    if (st != PAM_OK) return st;
    if ((st = check_prec(precision)) != PAM_OK) return st;
    const bool bf16 = precision == PAM_PREC_BF16;
    PAM_REQUIRE(params && x && target && mask && grads && B >= 1, "NULL argument or B < 1");
    PAM_CHECK_HIP(hipSetDevice(ctx->device));
    if ((st = ensure(ctx, BUF_CNN, cnn_ws_floats(B, true) * sizeof(float))) != PAM_OK) return st;
    const CnnWs w = carve(wsp<float>(ctx, BUF_CNN), B, true);
    KernelTimer kt(ctx, PAM_TK_CNN);
    forward(ctx, params, w, x, w.z, B, bf16);
    const int64_t nz = (int64_t)B * 2 * kPix;
    hipLaunchKernelGGL(k_bce, dim3(kBceBlocks), dim3(256), 0, ctx->stream, w.z, target, mask, nz, w.gz, w.bpart);
    hipLaunchKernelGGL(k_bce_scale, dim3(kBceBlocks), dim3(256), 0, ctx->stream, w.bpart, kBceBlocks, w.gz, nz,
                       loss);
    const int nblk = (B + kWgradPer - 1) / kWgradPer;
    const int nthin = (B + kWgradPerThin - 1) / kWgradPerThin;
    const float *act_in[4] = {x, w.a[0], w.a[1], w.a[2]};
    const float *gout = w.gz;
    for (int l = 3; l >= 0; --l) {
        const int nw = layer_size(l);
        int n_part = nblk;
        if (l == 3) {
            hipLaunchKernelGGL((k_wgrad<32, 2, 2, 8>), dim3(nthin), dim3(256), 0, ctx->stream, act_in[l], gout, B,
                               kWgradPerThin, w.part);
            n_part = nthin * 8;
        } else if (l == 0) {
            hipLaunchKernelGGL((k_wgrad<1, 32, 4, 16>), dim3(nthin), dim3(128), 0, ctx->stream, act_in[l], gout, B,
                               kWgradPerThin, w.part);
            n_part = nthin * 16;
        } else if (bf16) {
            n_part = (B + kWgradPer16 - 1) / kWgradPer16;
            hipLaunchKernelGGL(k_wgrad32_mfma, dim3(n_part), dim3(256), 0, ctx->stream, act_in[l], gout, B,
                               kWgradPer16, w.part);
        } else {
            hipLaunchKernelGGL((k_wgrad<32, 32, 4, 1>), dim3(nblk), dim3(256), 0, ctx->stream, act_in[l], gout, B,
                               kWgradPer, w.part);
        }
        hipLaunchKernelGGL(k_wgrad_reduce, dim3((nw + 63) / 64), dim3(256), 0, ctx->stream, w.part, n_part, nw,
                           grads + cnn_off(l));
        if (l == 0) break;
        // gradient of the layer input (a ReLU output): forward pass over the
        // flipped weights from cout to cin channels, gated by the activation
        float *gin = (gout == w.ga) ? w.gb : w.ga;
        if (bf16 && (l == 1 || l == 2))
            hipLaunchKernelGGL(k_conv32_mfma, dim3(mfma_grid(B)), dim3(256), 0, ctx->stream, gout,
                               w.hb + (size_t)(l - 1) * 32 * 32 * kTaps, (const float *)nullptr, gin, 2, act_in[l], B);
        else
            conv(ctx, cnn_cout(l), cnn_cin(l), gout, w.wb + cnn_off(l), nullptr, gin, B, 2, act_in[l]);
        gout = gin;
    }
    PAM_CHECK_HIP(hipGetLastError());
    return PAM_OK;
}

pam_status pam_cnn_adam(pam_ctx *ctx, float *params, const float *grads, float *m, float *v, int32_t step,
                        float lr, float beta1, float beta2, float eps) {
    pam_status st = check_ctx(ctx);
    if (st != PAM_OK) return st;
    PAM_REQUIRE(params && grads && m && v && step >= 1, "NULL argument or step < 1");
    PAM_REQUIRE(lr >= 0.0f && beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f,
                "Adam hyper-parameters out of range");
    PAM_CHECK_HIP(hipSetDevice(ctx->device));
    const float c1 = (float)(1.0 - pow((double)beta1, (double)step));
    const float c2 = (float)(1.0 - pow((double)beta2, (double)step));
    KernelTimer kt(ctx, PAM_TK_CNN);
    hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, ctx->stream, params, grads, m, v, kParams,
                       lr, beta1, beta2, eps, c1, c2);
    PAM_CHECK_HIP(hipGetLastError());
    return PAM_OK;
}

pam_status pam_grid_patches(pam_ctx *ctx, const pam_grid *grid, const double *cell_y, float scale,
                            int32_t *n_patches, float *patches) {
    pam_status st = check_ctx(ctx);
    if (st != PAM_OK) return st;
    std::vector<int32_t> tab;
    int np = 0, mx = 0;
    if ((st = patch_table(grid, tab, &np, &mx)) != PAM_OK) return st;
    PAM_REQUIRE(n_patches, "NULL n_patches");
    *n_patches = np;
    if (!patches) return PAM_OK;   // count query
    PAM_REQUIRE(cell_y, "NULL cell values");
    PAM_CHECK_HIP(hipSetDevice(ctx->device));
    const int n_sub = grid->n_sub[0] * grid->n_sub[1];
    if ((st = upload(ctx, BUF_TABLE, tab.data(), tab.size() * sizeof(int32_t))) != PAM_OK) return st;
    const int32_t *dt = wsp<int32_t>(ctx, BUF_TABLE);
    KernelTimer kt(ctx, PAM_TK_CNN);
    hipLaunchKernelGGL(k_patches, dim3(mx, n_sub), dim3(kPix), 0, ctx->stream, grid->n_cells[0], dt, dt + 4 * n_sub,
                       cell_y, scale, patches);
    PAM_CHECK_HIP(hipGetLastError());
    return PAM_OK;
}

pam_status pam_support_hint(pam_ctx *ctx, const pam_grid *grid, const pam_dict *dict, const float *logits,
                            float threshold, uint8_t *hint) {
    pam_status st = check_ctx(ctx);
    if (st != PAM_OK) return st;
    std::vector<int32_t> tab;
    int np = 0, mx = 0;
    if ((st = patch_table(grid, tab, &np, &mx)) != PAM_OK) return st;
    PAM_REQUIRE(dict && dict->dim == 2 && dict->m && dict->c && logits && hint, "NULL argument");
    const int n_sub = grid->n_sub[0] * grid->n_sub[1];
    PAM_REQUIRE(dict->n_sub == n_sub, "dictionary does not match the grid partition");
    PAM_REQUIRE(dict->m_cap >= 1, "m_cap < 1");
    PAM_CHECK_HIP(hipSetDevice(ctx->device));
    if ((st = upload(ctx, BUF_TABLE, tab.data(), tab.size() * sizeof(int32_t))) != PAM_OK) return st;
    const int32_t *dt = wsp<int32_t>(ctx, BUF_TABLE);
    const double h0 = (grid->hi[0] - grid->lo[0]) / grid->n_cells[0];
    const double h1 = (grid->hi[1] - grid->lo[1]) / grid->n_cells[1];
    KernelTimer kt(ctx, PAM_TK_CNN);
    hipLaunchKernelGGL(k_hint, dim3((dict->m_cap + 255) / 256, n_sub), dim3(256), 0, ctx->stream, dict->m_cap,
                       dict->m, dict->c, dt, dt + 4 * n_sub, grid->lo[0], grid->lo[1], h0, h1, logits, threshold, hint);
    PAM_CHECK_HIP(hipGetLastError());
    return PAM_OK;
}

pam_status pam_cnn_labels(pam_ctx *ctx, const pam_grid *grid, const pam_samples *samples, const pam_dict *dict,
                          const double *beta, const int32_t *elem_level, float *target, float *mask) {
    pam_status st = check_ctx(ctx);
    if (st != PAM_OK) return st;
    std::vector<int32_t> tab;
    int np = 0, mx = 0;
    if ((st = patch_table(grid, tab, &np, &mx)) != PAM_OK) return st;
    PAM_REQUIRE(samples && dict && beta && elem_level && target && mask && samples->off && samples->off_host &&
                    samples->x && dict->m && dict->c,
                "NULL argument");
    const int n_sub = grid->n_sub[0] * grid->n_sub[1];
    PAM_REQUIRE(dict->n_sub == n_sub && samples->n_sub == n_sub && dict->dim == 2 && samples->dim == 2,
                "samples / dictionary do not match the grid partition");
    PAM_REQUIRE(dict->m_cap >= 1, "m_cap < 1");
    int64_t n_max = 0;
    for (int s = 0; s < n_sub; ++s) n_max = std::max<int64_t>(n_max, samples->off_host[s + 1] - samples->off_host[s]);
    PAM_CHECK_HIP(hipSetDevice(ctx->device));
    if ((st = upload(ctx, BUF_TABLE, tab.data(), tab.size() * sizeof(int32_t))) != PAM_OK) return st;
    const int32_t *dt = wsp<int32_t>(ctx, BUF_TABLE);
    const double h0 = (grid->hi[0] - grid->lo[0]) / grid->n_cells[0];
    const double h1 = (grid->hi[1] - grid->lo[1]) / grid->n_cells[1];
    KernelTimer kt(ctx, PAM_TK_CNN);
    // every pixel starts unlabeled
    hipLaunchKernelGGL(k_fill, dim3((unsigned)std::min<int64_t>(((int64_t)np * 2 * kPix + 255) / 256, 65535)), dim3(256),
                       0, ctx->stream, mask, (int64_t)np * 2 * kPix, 0.0f);
    hipLaunchKernelGGL(k_fill, dim3((unsigned)std::min<int64_t>(((int64_t)np * 2 * kPix + 255) / 256, 65535)), dim3(256),
                       0, ctx->stream, target, (int64_t)np * 2 * kPix, 0.0f);
    const dim3 gc((dict->m_cap + 255) / 256, n_sub);
    for (int pass = 0; pass < 2; ++pass)
        hipLaunchKernelGGL(k_label_centers, gc, dim3(256), 0, ctx->stream, dict->m_cap, dict->m, dict->c, beta, dt,
                           dt + 4 * n_sub, grid->lo[0], grid->lo[1], h0, h1, pass, target, mask);
    if (n_max > 0)
        hipLaunchKernelGGL(k_label_samples, dim3((unsigned)((n_max + 255) / 256), n_sub), dim3(256), 0, ctx->stream,
                           samples->off, samples->x, elem_level, dt, dt + 4 * n_sub, grid->lo[0], grid->lo[1], h0, h1,
                           target, mask);
    PAM_CHECK_HIP(hipGetLastError());
    return PAM_OK;
}

}  // extern "C"
