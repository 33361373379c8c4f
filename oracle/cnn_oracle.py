"""FP64 CPU oracle of the learned warm start (a support prior for the cold
elastic-net fits; not a step of the paper's method).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product library. Plain numpy
in float64, written from the definitions:

* network: four 5x5 convolutions with zero padding 2 ("same" output size),
  1 -> 32 -> 32 -> 32 -> 2 channels, ReLU after the first three; parameters
  flattened per layer as w[cout][cin][5][5] then b[cout];
  conv(x)[b, o, i, j] = b[o] + sum_c sum_{u,v} w[o, c, u, v] x[b, c, i+u-2, j+v-2]
  (cross-correlation, as in the usual deep-learning convention);
* loss: binary cross-entropy with logits averaged over the masked entries;
* gradients: the chain rule taken layer by layer (no automatic
  differentiation); the pins check them against central differences;
* Adam (Kingma and Ba, 2015, Algorithm 1) with bias correction;
* optional emulation of the BF16 mode: the listed layers take their
  convolution operands rounded to bfloat16 (round to nearest even from the
  FP32 value), everything else in float64;
* the patch cut, the hint map and the training labels as index maps.
"""
from __future__ import annotations

import numpy as np

P = 16                     # patch side
K = 5                      # kernel side
CIN = (1, 32, 32, 32)
COUT = (32, 32, 32, 2)


def param_count() -> int:
    return sum(co * ci * K * K + co for ci, co in zip(CIN, COUT))


def unpack(params):
    """[(w [cout, cin, 5, 5], b [cout])] per layer, views into params."""
    params = np.asarray(params, np.float64)
    out, o = [], 0
    for ci, co in zip(CIN, COUT):
        w = params[o:o + co * ci * K * K].reshape(co, ci, K, K)
        o += co * ci * K * K
        b = params[o:o + co]
        o += co
        out.append((w, b))
    assert o == params.size
    return out


def bf16(a):
    """Round to bfloat16 (8-bit significand, round to nearest even) through
    float32, returned as float64."""
    u = np.ascontiguousarray(np.asarray(a, np.float64).astype(np.float32)).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------- network
def conv_same(x, w, b=None):
    """x [B, Ci, H, W], w [Co, Ci, 5, 5] -> [B, Co, H, W] (zero padding 2)."""
    Bn, Ci, H, W = x.shape
    xp = np.zeros((Bn, Ci, H + 4, W + 4))
    xp[:, :, 2:2 + H, 2:2 + W] = x
    out = np.zeros((Bn, w.shape[0], H, W))
    for u in range(K):
        for v in range(K):
            out += np.einsum("bchw,oc->bohw", xp[:, :, u:u + H, v:v + W], w[:, :, u, v])
    if b is not None:
        out += b[None, :, None, None]
    return out


def forward(params, x, bf16_layers=()):
    """logits [B, 2, 16, 16] and the per-layer inputs (for the backward pass).
    Layers in bf16_layers convolve BF16-rounded inputs and weights."""
    layers = unpack(params)
    a = np.asarray(x, np.float64).reshape(-1, 1, P, P)
    inputs = []
    for l, (w, b) in enumerate(layers):
        inputs.append(a)
        z = conv_same(bf16(a), bf16(w), b) if l in bf16_layers else conv_same(a, w, b)
        a = np.maximum(z, 0.0) if l < 3 else z
    return a, inputs


def bce(z, t, m):
    """Mean over the mask of max(z,0) - z t + log(1 + exp(-|z|)); d/dz."""
    z, t, m = (np.asarray(v, np.float64) for v in (z, t, m))
    cnt = m.sum()
    if cnt == 0:
        return 0.0, np.zeros_like(z)
    per = np.maximum(z, 0.0) - z * t + np.log1p(np.exp(-np.abs(z)))
    sig = 1.0 / (1.0 + np.exp(-z))
    return float((m * per).sum() / cnt), m * (sig - t) / cnt


def backward(params, inputs, dz, bf16_layers=()):
    """Gradient of the loss with respect to the flattened parameters, from
    d loss / d logits, by the chain rule through the four layers. Layers in
    bf16_layers take BF16-rounded operands in their weight-gradient and
    data-gradient products (the bias gradient sums the unrounded g)."""
    layers = unpack(params)
    grads = []
    g = np.asarray(dz, np.float64)             # gradient w.r.t. the layer output (pre-activation)
    for l in range(3, -1, -1):
        w, _ = layers[l]
        a = inputs[l]
        gb = g.sum(axis=(0, 2, 3))
        if l in bf16_layers:
            a, g, w = bf16(a), bf16(g), bf16(w)
        H = W = P
        ap = np.zeros((a.shape[0], a.shape[1], H + 4, W + 4))
        ap[:, :, 2:2 + H, 2:2 + W] = a
        gw = np.zeros_like(w)
        for u in range(K):
            for v in range(K):
                gw[:, :, u, v] = np.einsum("bohw,bchw->oc", g, ap[:, :, u:u + H, v:v + W])
        grads.append((gw, gb))
        if l == 0:
            break
        # d loss / d a[c, i, j] = sum_o sum_{u,v} w[o, c, u, v] g[o, i-u+2, j-v+2]
        gp = np.zeros((g.shape[0], g.shape[1], H + 4, W + 4))
        gp[:, :, 2:2 + H, 2:2 + W] = g
        ga = np.zeros_like(a)
        for u in range(K):
            for v in range(K):
                ga += np.einsum("bohw,oc->bchw", gp[:, :, 4 - u:4 - u + H, 4 - v:4 - v + W], w[:, :, u, v])
        g = ga * (inputs[l] > 0.0)             # through the ReLU that produced the input
    grads.reverse()
    return np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in grads])


def loss_grad(params, x, t, m, bf16_layers=()):
    z, inputs = forward(params, x, bf16_layers)
    loss, dz = bce(z, np.asarray(t).reshape(z.shape), np.asarray(m).reshape(z.shape))
    return loss, backward(params, inputs, dz, bf16_layers)


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step; returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------- index maps
def owned_boxes_cells(grid):
    """(i0, j0, ni, nj) per subdomain of a 2-D grid, axis 0 fastest."""
    b0, b1 = np.asarray(grid.breaks[0]), np.asarray(grid.breaks[1])
    out = []
    for k1 in range(grid.n_sub[1]):
        for k0 in range(grid.n_sub[0]):
            out.append((int(b0[k0]), int(b1[k1]), int(b0[k0 + 1] - b0[k0]), int(b1[k1 + 1] - b1[k1])))
    return out


def patch_index(grid):
    """First patch index of every subdomain and the total count."""
    base, tot = [], 0
    for (_, _, ni, nj) in owned_boxes_cells(grid):
        base.append(tot)
        tot += (ni // P) * (nj // P)
    return base, tot


def patches(grid, scale):
    """[n_patches, 16, 16] float32 of float64(scale) * y, per subdomain
    row-major over its patch grid (axis 0 fastest)."""
    Y = np.asarray(grid.y, np.float64).reshape(grid.n_cells[1], grid.n_cells[0])
    out = []
    for (i0, j0, ni, nj) in owned_boxes_cells(grid):
        for pj in range(nj // P):
            for pi in range(ni // P):
                blk = Y[j0 + pj * P:j0 + (pj + 1) * P, i0 + pi * P:i0 + (pi + 1) * P]
                out.append((np.float64(scale) * blk).astype(np.float32))
    return np.stack(out)


def _cell_of(grid, box, x0, x1):
    """Owned-box-local cell of a point: floor((x - lo) / h) clamped."""
    i0, j0, ni, nj = box
    h0 = (grid.hi[0] - grid.lo[0]) / grid.n_cells[0]
    h1 = (grid.hi[1] - grid.lo[1]) / grid.n_cells[1]
    ix = int(np.floor((x0 - grid.lo[0]) / h0)) - i0
    iy = int(np.floor((x1 - grid.lo[1]) / h1)) - j0
    return ix, iy


def _pixel(box, base, ix, iy):
    ni = box[2]
    return base + (iy // P) * (ni // P) + ix // P, iy % P, ix % P


def hint(grid, m, c, m_cap, logits, thr):
    """uint8 [n_sub, m_cap]: support logit of the cell holding each center > thr."""
    boxes = owned_boxes_cells(grid)
    base, _ = patch_index(grid)
    logits = np.asarray(logits).reshape(-1, 2, P, P)
    c = np.asarray(c).reshape(len(boxes), m_cap, 2)
    out = np.zeros((len(boxes), m_cap), np.uint8)
    for s, box in enumerate(boxes):
        for k in range(int(m[s])):
            ix, iy = _cell_of(grid, box, c[s, k, 0], c[s, k, 1])
            ix = min(max(ix, 0), box[2] - 1)
            iy = min(max(iy, 0), box[3] - 1)
            p, r, q = _pixel(box, base[s], ix, iy)
            out[s, k] = 1 if logits[p, 1, r, q] > thr else 0
    return out


def labels(grid, off, x, m, c, m_cap, beta, elem_level):
    """(target, mask) [n_patches, 2, 16, 16] float32: channel 1 from the
    centers (any active center in a cell -> 1), channel 0 from the owned
    samples (elem_level > 0 -> 1)."""
    boxes = owned_boxes_cells(grid)
    base, tot = patch_index(grid)
    t = np.zeros((tot, 2, P, P), np.float32)
    mk = np.zeros((tot, 2, P, P), np.float32)
    c = np.asarray(c).reshape(len(boxes), m_cap, 2)
    beta = np.asarray(beta).reshape(len(boxes), m_cap)
    x = np.asarray(x).reshape(-1, 2)
    for s, box in enumerate(boxes):
        for k in range(int(m[s])):
            ix, iy = _cell_of(grid, box, c[s, k, 0], c[s, k, 1])
            ix = min(max(ix, 0), box[2] - 1)
            iy = min(max(iy, 0), box[3] - 1)
            p, r, q = _pixel(box, base[s], ix, iy)
            mk[p, 1, r, q] = 1.0
            if beta[s, k] != 0.0:
                t[p, 1, r, q] = 1.0
        for j in range(int(off[s]), int(off[s + 1])):
            ix, iy = _cell_of(grid, box, x[j, 0], x[j, 1])
            if 0 <= ix < box[2] and 0 <= iy < box[3]:
                p, r, q = _pixel(box, base[s], ix, iy)
                mk[p, 0, r, q] = 1.0
                t[p, 0, r, q] = 1.0 if elem_level[j] > 0 else 0.0
    return t, mk
