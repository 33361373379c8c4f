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
