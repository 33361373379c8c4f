"""Learned warm start: training data from the method's own fits, training,
and the support hint for cold fits. Every step runs in libpam.so (patches,
labels, network forward/backward, Adam, hint map); this module sequences
the calls."""
from __future__ import annotations

from typing import Sequence

import numpy as np
import torch

from . import api
from .synth import CNN_SCALE


def labelled_patches(ctx: api.Context, grid, g: Sequence[int], k_top: int, opts: api.EnetOpts,
                     eps_tol: float):
    """(patches, target, mask) of one 2-D grid: support labels from the cold
    fit on the initial lattice, refinement labels from the elements the first
    round of Alg. 1 marks."""
    S = api.partition(ctx, grid)
    m0 = int(np.prod(g[: grid.dim]))
    D = api.init_lattice(ctx, grid, g, m_cap=m0 + (2 ** grid.dim - 1) * k_top)
    beta, _ = api.fit(ctx, S, D, opts)
    D1 = D.clone()
    _, lvl, _, _, _ = api.refine(ctx, S, D1, opts, api.RefineOpts(k_top=k_top, max_rounds=1,
                                                                   eps_tol=eps_tol),
                                 beta=beta.clone())
    t, m = api.cnn_labels(ctx, grid, S, D, beta, lvl)
    x = api.grid_patches(ctx, grid, scale=CNN_SCALE)
    return x, t, m


def training_set(ctx: api.Context, grids, g, k_top, opts, eps_tol_rel=1e-4):
    xs, ts, ms = [], [], []
    for grid in grids:
        cell = np.prod([(grid.hi[a] - grid.lo[a]) / grid.n_cells[a] for a in range(grid.dim)])
        x, t, m = labelled_patches(ctx, grid, g, k_top, opts, eps_tol_rel * cell)
        xs.append(x)
        ts.append(t)
        ms.append(m)
    return torch.cat(xs), torch.cat(ts), torch.cat(ms)


def hint(ctx: api.Context, params: torch.Tensor, grid, D: api.Dictionary, threshold: float = 0.0,
         precision: str = "f32"):
    """uint8 [n_sub, m_cap] support hint of the trained network for D on grid."""
    z = api.cnn_forward(ctx, params, api.grid_patches(ctx, grid, scale=CNN_SCALE), precision)
    return api.support_hint(ctx, grid, D, z, threshold)


def head_accuracy(logits: torch.Tensor, target: torch.Tensor, mask: torch.Tensor):
    """Per channel: (accuracy at p > 1/2, accuracy of the constant majority
    guess, labelled count) over the masked cells."""
    out = []
    for ch in range(2):
        mk = mask[:, ch] > 0
        n = int(mk.sum())
        if n == 0:
            out.append((float("nan"), float("nan"), 0))
            continue
        pred = logits[:, ch][mk] > 0
        tg = target[:, ch][mk] > 0.5
        pos = float(tg.float().mean())
        out.append((float((pred == tg).float().mean()), max(pos, 1.0 - pos), n))
    return out


def _throughput(B: int = 1024, steps: int = 10):
    """Loss-and-gradient plus Adam steps on seeded patches, both precisions:
    prints patches/s and the network's FLOP rate (fwd 27.4 MFLOP per patch,
    training about 3x)."""
    import time
    from . import synth
    ctx = api.Context(0)
    p = api.cnn_init(1, 0)
    x, t, m = (torch.as_tensor(a, device="cuda") for a in synth.cnn_batch(2, B))
    f_fwd = 2.0 * 256 * 25 * (1 * 32 + 32 * 32 + 32 * 32 + 32 * 2)
    g = torch.empty_like(p)
    mom, var = torch.zeros_like(p), torch.zeros_like(p)
    for prec in ("f32", "bf16"):
        api.cnn_loss_grad(ctx, p, x, t, m, g, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            api.cnn_loss_grad(ctx, p, x, t, m, g, precision=prec)
            api.cnn_adam(ctx, p, g, mom, var, k + 1, 1e-4)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        print(f"{prec}: B={B} {dt * 1e3:.2f} ms per training step, {B / dt:.0f} patches/s, "
              f"{3 * f_fwd * B / dt / 1e12:.1f} TFLOP/s", flush=True)
    ctx.close()


if __name__ == "__main__":
    _throughput()
