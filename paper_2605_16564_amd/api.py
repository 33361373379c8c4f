"""Torch-facing wrappers of the C ABI: device buffers come from torch, every
step of the method runs in libpam.so (see native.py). No CPU fallback."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import native as N


def _p(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _require_cuda(t: torch.Tensor, name: str):
    if not t.is_cuda:
        raise N.PamError(f"{name} must be a device tensor")


class Context:
    """One pam_ctx bound to a device; work goes on torch's current stream."""

    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise N.PamError("no HIP device available")
        self.device = device
        h = C.c_void_p()
        N.check(N.lib().pam_create(C.byref(h), device), "pam_create")
        self.h = h
        self.use_current_stream()

    def use_current_stream(self):
        s = torch.cuda.current_stream(self.device)
        N.check(N.lib().pam_set_stream(self.h, C.c_void_p(s.cuda_stream)), "pam_set_stream")

    def sync(self):
        N.check(N.lib().pam_sync(self.h), "pam_sync")

    def graphs(self, on: bool = True):
        """Fits and refinements as one HIP graph launch each (default on)."""
        N.check(N.lib().pam_graph_enable(self.h, 1 if on else 0), "pam_graph_enable")

    def gram_path(self, mode: str = "tuned"):
        """FP32/BF16 Gram path: 'tuned' (default), 'materialized' or 'fused'."""
        m = {"tuned": 0, "materialized": 1, "fused": 2}[mode]
        N.check(N.lib().pam_gram_path(self.h, m), "pam_gram_path")

    def timing(self, on: bool = True):
        N.check(N.lib().pam_timing_enable(self.h, 1 if on else 0), "pam_timing_enable")

    def timing_read(self, reset: bool = True):
        """{kernel kind: (total ms, launches)} since the last reset."""
        k = len(N.TIMING_KINDS)
        ms = np.zeros(k)
        cnt = np.zeros(k, np.int64)
        N.check(N.lib().pam_timing_read(self.h, ms.ctypes.data_as(C.c_void_p),
                                        cnt.ctypes.data_as(C.c_void_p), 1 if reset else 0),
                "pam_timing_read")
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(N.TIMING_KINDS)}

    def close(self):
        if self.h:
            N.lib().pam_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- a1
def _grid_struct(grid):
    d = grid.dim
    g = N.PamGrid()
    g.dim = d
    brk = np.ascontiguousarray(np.concatenate([np.asarray(b, np.int32) for b in grid.breaks[:d]]),
                               dtype=np.int32)
    for a in range(3):
        g.n_cells[a] = int(grid.n_cells[a]) if a < d else 1
        g.n_sub[a] = int(grid.n_sub[a]) if a < d else 1
        g.lo[a] = float(grid.lo[a]) if a < d else 0.0
        g.hi[a] = float(grid.hi[a]) if a < d else 1.0
    g.breaks = brk.ctypes.data_as(C.c_void_p)
    g.overlap = float(grid.overlap)
    return g, brk  # keep brk alive


@dataclass
class Samples:
    dim: int
    n_sub: int
    n_max: int
    off: torch.Tensor       # int64 [n_sub+1] device
    off_host: np.ndarray    # int64 [n_sub+1]
    x: torch.Tensor         # f64 [N_tot, dim]
    y: torch.Tensor         # f64 [N_tot]
    h: torch.Tensor         # f64 [N_tot, dim]
    cell: Optional[torch.Tensor] = None

    def struct(self):
        s = N.PamSamples()
        s.dim, s.n_sub, s.n_max = self.dim, self.n_sub, self.n_max
        s.off = _p(self.off)
        s.off_host = self.off_host.ctypes.data_as(C.c_void_p)
        s.x, s.y, s.h = _p(self.x), _p(self.y), _p(self.h)
        return s


def concat_samples(parts: Sequence[Samples]) -> Samples:
    """Samples of several grids as one batch (subdomains in order)."""
    off = [np.zeros(1, np.int64)]
    base = 0
    for S in parts:
        off.append(S.off_host[1:] + base)
        base += int(S.off_host[-1])
    off_h = np.concatenate(off)
    dev = parts[0].x.device
    return Samples(parts[0].dim, int(sum(S.n_sub for S in parts)), int(max(S.n_max for S in parts)),
                   torch.as_tensor(off_h, device=dev), off_h, torch.cat([S.x for S in parts]),
                   torch.cat([S.y for S in parts]), torch.cat([S.h for S in parts]),
                   torch.cat([S.cell for S in parts]) if all(S.cell is not None for S in parts) else None)


def partition_count(grid):
    g, brk = _grid_struct(grid)
    n = int(np.prod(grid.n_sub[: grid.dim]))
    off = np.zeros(n + 1, np.int64)
    nmax = C.c_int32()
    N.check(N.lib().pam_partition_count(C.byref(g), off.ctypes.data_as(C.c_void_p), C.byref(nmax)),
            "pam_partition_count")
    return off, int(nmax.value)


def partition(ctx: Context, grid, cell_y: Optional[torch.Tensor] = None) -> Samples:
    """a1: samples of every subdomain, gathered on the device."""
    dev = torch.device("cuda", ctx.device)
    off, nmax = partition_count(grid)
    d = grid.dim
    tot = int(off[-1])
    if cell_y is None:
        cell_y = torch.as_tensor(np.ascontiguousarray(grid.y, np.float64), device=dev)
    _require_cuda(cell_y, "cell_y")
    off_d = torch.as_tensor(off, device=dev)
    x = torch.empty((tot, d), dtype=torch.float64, device=dev)
    y = torch.empty(tot, dtype=torch.float64, device=dev)
    h = torch.empty((tot, d), dtype=torch.float64, device=dev)
    cell = torch.empty((tot, d), dtype=torch.int32, device=dev)
    g, brk = _grid_struct(grid)
    ctx.use_current_stream()
    N.check(N.lib().pam_partition_gather(ctx.h, C.byref(g), _p(cell_y), _p(off_d), _p(x), _p(y),
                                         _p(h), _p(cell)), "pam_partition_gather")
    n = int(np.prod(grid.n_sub[:d]))
    return Samples(d, n, nmax, off_d, off, x, y, h, cell)


# ---------------------------------------------------------------- dictionary
@dataclass
class Dictionary:
    n_sub: int
    dim: int
    m_cap: int
    m: torch.Tensor        # int32 [n_sub]
    c: torch.Tensor        # f64 [n_sub, m_cap, dim]
    sigma: torch.Tensor    # f64 [n_sub, m_cap]
    level: torch.Tensor    # int32 [n_sub, m_cap]
    basis: str = "shepard" # "shepard" (the method's) or "plain" (the unnormalized ablation)

    @staticmethod
    def empty(n_sub, dim, m_cap, device):
        dev = torch.device("cuda", device) if isinstance(device, int) else device
        return Dictionary(n_sub, dim, m_cap,
                          torch.zeros(n_sub, dtype=torch.int32, device=dev),
                          torch.zeros((n_sub, m_cap, dim), dtype=torch.float64, device=dev),
                          torch.ones((n_sub, m_cap), dtype=torch.float64, device=dev),
                          torch.zeros((n_sub, m_cap), dtype=torch.int32, device=dev))

    def clone(self):
        return Dictionary(self.n_sub, self.dim, self.m_cap, self.m.clone(), self.c.clone(),
                          self.sigma.clone(), self.level.clone(), self.basis)

    def struct(self):
        s = N.PamDict()
        s.n_sub, s.dim, s.m_cap = self.n_sub, self.dim, self.m_cap
        s.m, s.c, s.sigma, s.level = _p(self.m), _p(self.c), _p(self.sigma), _p(self.level)
        if self.basis not in N.BASIS:
            raise N.PamError("basis must be 'shepard' or 'plain'")
        s.basis = N.BASIS[self.basis]
        return s


def concat_dicts(parts: Sequence["Dictionary"]) -> "Dictionary":
    """Dictionaries of several grids (same dim and m_cap) as one batch."""
    d0 = parts[0]
    if any(D.m_cap != d0.m_cap or D.dim != d0.dim or D.basis != d0.basis for D in parts):
        raise N.PamError("dictionaries to concatenate need the same dim, m_cap and basis")
    return Dictionary(int(sum(D.n_sub for D in parts)), d0.dim, d0.m_cap, torch.cat([D.m for D in parts]),
                      torch.cat([D.c for D in parts]), torch.cat([D.sigma for D in parts]),
                      torch.cat([D.level for D in parts]), d0.basis)


def init_lattice(ctx: Context, grid, g: Sequence[int], m_cap: int, sigma_factor: float = 1.0,
                 basis: str = "shepard"):
    """a2: g^d lattice dictionary per owned box (basis: "shepard", the method's
    normalized functions, or "plain", the unnormalized Gaussians)."""
    D = Dictionary.empty(int(np.prod(grid.n_sub[: grid.dim])), grid.dim, m_cap, ctx.device)
    D.basis = basis
    gs, brk = _grid_struct(grid)
    garr = np.ascontiguousarray(np.asarray(g[: grid.dim], np.int32))
    ds = D.struct()
    ctx.use_current_stream()
    N.check(N.lib().pam_init_lattice(ctx.h, C.byref(gs), garr.ctypes.data_as(C.c_void_p),
                                     float(sigma_factor), C.byref(ds)), "pam_init_lattice")
    return D


# ---------------------------------------------------------------- a3-a9
@dataclass
class EnetOpts:
    lambda1: float
    lambda2: float
    precision: str = "f64"
    cd_sweeps: int = 8
    max_iter: int = 100000
    batched: bool = True
    lambda1_sub: Optional[torch.Tensor] = None
    lambda2_sub: Optional[torch.Tensor] = None
    support_hint: Optional[torch.Tensor] = None
    team: int = 0          # workgroups per subdomain in the solve (0 auto, 1, 2, 4)
    team_min: int = 0      # active-set size from which a team shares passes (0: 128)
    team_idle_us: int = 0  # a member's wait for the next pass before it leaves (0: 10 s)

    def struct(self, warm_start: bool):
        o = N.PamEnetOpts()
        o.lambda1, o.lambda2 = float(self.lambda1), float(self.lambda2)
        o.lambda1_sub, o.lambda2_sub = _p(self.lambda1_sub), _p(self.lambda2_sub)
        o.precision = N.PREC[self.precision]
        o.cd_sweeps, o.max_iter = int(self.cd_sweeps), int(self.max_iter)
        o.warm_start = 1 if warm_start else 0
        o.batched = 1 if self.batched else 0
        o.support_hint = _p(self.support_hint)
        o.team, o.team_min, o.team_idle_us = int(self.team), int(self.team_min), int(self.team_idle_us)
        return o


STATS_DTYPE = np.dtype([("status", np.int32), ("cd_sweeps", np.int32), ("iters", np.int32),
                        ("support", np.int32), ("kkt", np.float64),
                        ("stream_bytes", np.float64), ("polish", np.int32),
                        ("team", np.int32), ("solve_us", np.float64)])


def new_stats(n_sub, device):
    return torch.zeros(n_sub * N.STATS_BYTES, dtype=torch.uint8,
                       device=torch.device("cuda", device) if isinstance(device, int) else device)


def stats_to_numpy(stats: torch.Tensor) -> np.ndarray:
    return stats.cpu().numpy().view(STATS_DTYPE)


def fit(ctx: Context, S: Samples, D: Dictionary, opts: EnetOpts,
        beta: Optional[torch.Tensor] = None, stats: Optional[torch.Tensor] = None,
        warm: Optional[bool] = None):
    """a3-a6 for every subdomain; returns (beta [n_sub, m_cap] f64, stats tensor).
    warm: beta holds the starting point (default: when beta is given)."""
    warm = (beta is not None) if warm is None else warm
    if beta is None:
        beta = torch.zeros((D.n_sub, D.m_cap), dtype=torch.float64, device=D.m.device)
    if stats is None:
        stats = new_stats(D.n_sub, D.m.device)
    ss, ds, os_ = S.struct(), D.struct(), opts.struct(warm)
    ctx.use_current_stream()
    N.check(N.lib().pam_fit_subdomains(ctx.h, C.byref(ss), C.byref(ds), C.byref(os_), _p(beta),
                                       _p(stats)), "pam_fit_subdomains")
    return beta, stats


def refit_nonconverged(ctx: Context, S: Samples, D: Dictionary, opts: EnetOpts, beta: torch.Tensor,
                       stats: torch.Tensor):
    """a3-a6 with the FP64 Gram, cold, for the subdomains whose stats read
    not converged (the previous fit's beta and stats, updated in place)."""
    ss, ds, os_ = S.struct(), D.struct(), opts.struct(False)
    ctx.use_current_stream()
    N.check(N.lib().pam_refit_nonconverged(ctx.h, C.byref(ss), C.byref(ds), C.byref(os_), _p(beta),
                                           _p(stats)), "pam_refit_nonconverged")
    return beta, stats


def select_lambda(ctx: Context, S: Samples, D: Dictionary, opts: EnetOpts, n_alpha: int = 8,
                  k_folds: int = 5, alpha_min_ratio: float = 1e-3, l1_ratio: float = 0.99):
    """Per-subdomain elastic-net parameters by an alpha path and K-fold
    cross-validation (opts gives the precision and iteration controls).
    Returns dict of device tensors: alpha and score [n_sub, n_alpha], best
    [n_sub], lambda1 and lambda2 [n_sub] (for EnetOpts.lambda1_sub/_sub),
    n_failed [n_sub]."""
    dev = D.m.device
    n = D.n_sub
    out = dict(alpha=torch.empty((n, n_alpha), dtype=torch.float64, device=dev),
               score=torch.empty((n, n_alpha), dtype=torch.float64, device=dev),
               best=torch.empty(n, dtype=torch.int32, device=dev),
               lambda1=torch.empty(n, dtype=torch.float64, device=dev),
               lambda2=torch.empty(n, dtype=torch.float64, device=dev),
               n_failed=torch.empty(n, dtype=torch.int32, device=dev))
    sel = N.PamSelectOpts()
    sel.n_alpha, sel.k_folds = int(n_alpha), int(k_folds)
    sel.alpha_min_ratio, sel.l1_ratio = float(alpha_min_ratio), float(l1_ratio)
    ss, ds, os_ = S.struct(), D.struct(), opts.struct(False)
    ctx.use_current_stream()
    N.check(N.lib().pam_select_lambda(ctx.h, C.byref(ss), C.byref(ds), C.byref(os_), C.byref(sel),
                                      _p(out["alpha"]), _p(out["score"]), _p(out["best"]),
                                      _p(out["lambda1"]), _p(out["lambda2"]), _p(out["n_failed"])),
            "pam_select_lambda")
    return out


@dataclass
class RefineOpts:
    k_top: int = 204
    k_top_sub: Optional[np.ndarray] = None
    max_rounds: int = 3
    m_max: int = 1 << 30
    eta: float = 0.5
    eps_tol: float = 0.0
    space: int = 0
    cold_rounds: bool = False


def refine(ctx: Context, S: Samples, D: Dictionary, opts: EnetOpts, ropts: RefineOpts,
           beta: Optional[torch.Tensor] = None, elem_level: Optional[torch.Tensor] = None,
           out: Optional[dict] = None, warm: Optional[bool] = None):
    """Alg. 1 on every subdomain (D is updated in place).
    Returns (beta, elem_level, rounds, round_stats [n_sub, R+1, 7], stats).
    out: optional dict of caller-owned outputs (rounds, round_stats, stats)
    reused instead of new tensors; warm: beta is a warm start (default: when
    beta is given)."""
    dev = D.m.device
    warm = (beta is not None) if warm is None else warm
    if beta is None:
        beta = torch.zeros((D.n_sub, D.m_cap), dtype=torch.float64, device=dev)
    if elem_level is None:
        elem_level = torch.zeros(int(S.off_host[-1]), dtype=torch.int32, device=dev)
    out = out or {}
    rounds = out.get("rounds")
    if rounds is None:
        rounds = torch.zeros(D.n_sub, dtype=torch.int32, device=dev)
    rstats = out.get("round_stats")
    if rstats is None:
        rstats = torch.zeros((D.n_sub, ropts.max_rounds + 1, 7), dtype=torch.float64, device=dev)
    stats = out.get("stats")
    if stats is None:
        stats = new_stats(D.n_sub, dev)
    r = N.PamRefineOpts()
    r.k_top = int(ropts.k_top)
    kts = None
    if ropts.k_top_sub is not None:
        kts = np.ascontiguousarray(ropts.k_top_sub, dtype=np.int32)
        r.k_top_sub = kts.ctypes.data_as(C.c_void_p)
    r.max_rounds, r.m_max = int(ropts.max_rounds), int(min(ropts.m_max, 2 ** 31 - 1))
    r.eta, r.eps_tol, r.space = float(ropts.eta), float(ropts.eps_tol), int(ropts.space)
    r.elem_level, r.rounds, r.round_stats = _p(elem_level), _p(rounds), _p(rstats)
    r.cold_rounds = 1 if ropts.cold_rounds else 0
    ss, ds, os_ = S.struct(), D.struct(), opts.struct(warm)
    ctx.use_current_stream()
    N.check(N.lib().pam_refine(ctx.h, C.byref(ss), C.byref(ds), _p(beta), C.byref(os_),
                               C.byref(r), _p(stats)), "pam_refine")
    return beta, elem_level, rounds, rstats, stats


# ---------------------------------------------------------------- a10
def axis_coords(grid) -> List[np.ndarray]:
    out = []
    for a in range(grid.dim):
        hcell = (grid.hi[a] - grid.lo[a]) / grid.n_cells[a]
        out.append(np.array([grid.lo[a] + float(b) * hcell for b in grid.breaks[a]]))
    return out


def _field_table(grids, Q, q_counts, sub_bases):
    """pam_field array (and the breakpoint arrays it points into) for one or
    several fields whose subdomains are concatenated in one dictionary."""
    if q_counts is None:
        q_counts = [Q]
    if sub_bases is None:
        sub_bases, acc = [], 0
        for g in grids:
            sub_bases.append(acc)
            acc += int(np.prod(g.n_sub[: g.dim]))
    fields = (N.PamField * len(grids))()
    keep = []
    q0 = 0
    for f, g in enumerate(grids):
        ax = np.ascontiguousarray(np.concatenate(axis_coords(g)), dtype=np.float64)
        keep.append(ax)
        F = fields[f]
        F.dim = g.dim
        for a in range(3):
            F.n_sub_axis[a] = int(g.n_sub[a]) if a < g.dim else 1
        F.axis_x = ax.ctypes.data_as(C.c_void_p)
        F.sub_base = int(sub_bases[f])
        F.q_begin, F.q_end = q0, q0 + int(q_counts[f])
        q0 += int(q_counts[f])
    return fields, keep


def _query_dtype(xq: torch.Tensor) -> int:
    _require_cuda(xq, "xq")
    if xq.dtype not in (torch.float32, torch.float64):
        raise N.PamError("xq must be float32 or float64")
    return 0 if xq.dtype == torch.float32 else 1


def evaluate(ctx: Context, grids, D: Dictionary, beta: torch.Tensor, xq: torch.Tensor,
             q_counts: Optional[Sequence[int]] = None, sub_bases: Optional[Sequence[int]] = None,
             space: int = 0, n_outside: Optional[torch.Tensor] = None) -> torch.Tensor:
    """K*(x) of one or several fields (subdomains concatenated in D) at xq.
    xq is float32 or float64 [Q, dim]; field f owns q_counts[f] consecutive rows."""
    if not isinstance(grids, (list, tuple)):
        grids = [grids]
    dtype = _query_dtype(xq)
    Q = int(xq.shape[0])
    fields, keep = _field_table(grids, Q, q_counts, sub_bases)
    out = torch.empty(Q, dtype=xq.dtype, device=xq.device)
    ds = D.struct()
    ctx.use_current_stream()
    N.check(N.lib().pam_eval(ctx.h, len(grids), fields, C.byref(ds), _p(beta), dtype,
                             _p(xq.contiguous()), Q, _p(out), int(space), _p(n_outside)),
            "pam_eval")
    return out


def evaluate_noalloc(ctx: Context, grids, D: Dictionary, beta: torch.Tensor, xq: torch.Tensor,
                     out: torch.Tensor, q_counts: Optional[Sequence[int]] = None,
                     sub_bases: Optional[Sequence[int]] = None, space: int = 0,
                     n_outside: Optional[torch.Tensor] = None) -> torch.Tensor:
    """evaluate() through pam_eval_noalloc: the library allocates nothing
    (fixed per-device scratch); the caller passes the output buffer."""
    if not isinstance(grids, (list, tuple)):
        grids = [grids]
    dtype = _query_dtype(xq)
    Q = int(xq.shape[0])
    if out.dtype != xq.dtype or out.numel() < Q or not out.is_cuda:
        raise N.PamError("out must be a device tensor of the query dtype with Q entries")
    fields, keep = _field_table(grids, Q, q_counts, sub_bases)
    ds = D.struct()
    ctx.use_current_stream()
    N.check(N.lib().pam_eval_noalloc(ctx.h, len(grids), fields, C.byref(ds), _p(beta), dtype,
                                     _p(xq.contiguous()), Q, _p(out), int(space), _p(n_outside)),
            "pam_eval_noalloc")
    return out


def evaluate_blend(ctx: Context, grids, D: Dictionary, beta: torch.Tensor, xq: torch.Tensor,
                   blend: float, q_counts: Optional[Sequence[int]] = None,
                   sub_bases: Optional[Sequence[int]] = None, space: int = 0,
                   n_outside: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Continuous reconstruction: neighbouring local surrogates averaged over
    interface bands of half-width blend * (shorter neighbouring interval).
    Arguments as evaluate; blend = 0 gives evaluate's result exactly."""
    if not isinstance(grids, (list, tuple)):
        grids = [grids]
    dtype = _query_dtype(xq)
    Q = int(xq.shape[0])
    fields, keep = _field_table(grids, Q, q_counts, sub_bases)
    out = torch.empty(Q, dtype=xq.dtype, device=xq.device)
    ds = D.struct()
    ctx.use_current_stream()
    N.check(N.lib().pam_eval_blend(ctx.h, len(grids), fields, C.byref(ds), _p(beta), float(blend),
                                   dtype, _p(xq.contiguous()), Q, _p(out), int(space),
                                   _p(n_outside)),
            "pam_eval_blend")
    return out


def interface_count(grids) -> int:
    if not isinstance(grids, (list, tuple)):
        grids = [grids]
    fields, keep = _field_table(grids, 0, [0] * len(grids), None)
    return int(N.lib().pam_interface_count(len(grids), fields))


def interface_jump(ctx: Context, grids, D: Dictionary, beta: torch.Tensor, n_per_axis: int,
                   sub_bases: Optional[Sequence[int]] = None) -> torch.Tensor:
    """float64 [n_interfaces, 2]: (max, mean) |K*_A - K*_B| on every interior
    interface piece, ordered by field, axis, then upper subdomain."""
    if not isinstance(grids, (list, tuple)):
        grids = [grids]
    fields, keep = _field_table(grids, 0, [0] * len(grids), sub_bases)
    nf = int(N.lib().pam_interface_count(len(grids), fields))
    if nf < 0:
        raise N.PamError("bad field table")
    out = torch.empty((max(nf, 1), 2), dtype=torch.float64, device=beta.device)
    ds = D.struct()
    ctx.use_current_stream()
    N.check(N.lib().pam_interface_jump(ctx.h, len(grids), fields, C.byref(ds), _p(beta),
                                       int(n_per_axis), _p(out)), "pam_interface_jump")
    return out[:nf]


# ---------------------------------------------------------------- Darcy consumer
@dataclass
class DarcyOpts:
    n0: int
    n1: int
    lo: Sequence[float] = (0.0, 0.0)
    hi: Sequence[float] = (1.0, 1.0)
    p_left: float = 1.0
    p_right: float = 0.0
    tol: float = 1e-10
    max_iter: int = 200000
    check_every: int = 64

    def struct(self):
        o = N.PamDarcyOpts()
        o.n[0], o.n[1] = int(self.n0), int(self.n1)
        for a in range(2):
            o.lo[a], o.hi[a] = float(self.lo[a]), float(self.hi[a])
        o.p_left, o.p_right, o.tol = float(self.p_left), float(self.p_right), float(self.tol)
        o.max_iter, o.check_every = int(self.max_iter), int(self.check_every)
        return o


def darcy_k_from_reconstruction(ctx: Context, grid, D: Dictionary, beta: torch.Tensor,
                                o: DarcyOpts, blend: Optional[float] = None) -> torch.Tensor:
    """K = 10^K* at the triangle centroids (owner reconstruction, or the
    continuous one with the given band), float64 [n1, n0, 2] on the device."""
    k = torch.empty((o.n1, o.n0, 2), dtype=torch.float64, device=beta.device)
    fields, keep = _field_table([grid], 0, None, None)
    os_, ds = o.struct(), D.struct()
    ctx.use_current_stream()
    N.check(N.lib().pam_darcy_coefficient(ctx.h, C.byref(os_), fields, C.byref(ds), _p(beta),
                                          -1.0 if blend is None else float(blend), _p(k)),
            "pam_darcy_coefficient")
    del keep
    return k


def darcy_k_from_cells(ctx: Context, grid, o: DarcyOpts) -> torch.Tensor:
    """The data's own coefficient 10^y on a mesh whose squares are the data
    cells (n0, n1 = the grid's cells): both triangles of a square take it."""
    if (o.n0, o.n1) != (grid.n_cells[0], grid.n_cells[1]):
        raise N.PamError("the mesh must be the data grid")
    y = torch.as_tensor(grid.y, dtype=torch.float64, device="cuda")
    k = torch.empty((o.n1, o.n0, 2), dtype=torch.float64, device=y.device)
    os_ = o.struct()
    ctx.use_current_stream()
    N.check(N.lib().pam_darcy_coefficient_cells(ctx.h, C.byref(os_), _p(y), _p(k)),
            "pam_darcy_coefficient_cells")
    return k


def darcy_solve(ctx: Context, o: DarcyOpts, k_tri: torch.Tensor, p: Optional[torch.Tensor] = None):
    """Nodal pressure (float64 [(n1+1)(n0+1)]), iterations, final relative residual."""
    _require_cuda(k_tri, "k_tri")
    warm = p is not None
    if p is None:
        p = torch.empty((o.n0 + 1) * (o.n1 + 1), dtype=torch.float64, device=k_tri.device)
    it = C.c_int32(0)
    res = C.c_double(0.0)
    os_ = o.struct()
    ctx.use_current_stream()
    N.check(N.lib().pam_darcy_solve(ctx.h, C.byref(os_), _p(k_tri.contiguous()), _p(p),
                                    1 if warm else 0, C.byref(it), C.byref(res)), "pam_darcy_solve")
    return p, int(it.value), float(res.value)


def darcy_error(ctx: Context, o: DarcyOpts, p_ref: torch.Tensor, p: torch.Tensor) -> float:
    e = C.c_double(0.0)
    os_ = o.struct()
    ctx.use_current_stream()
    N.check(N.lib().pam_darcy_error(ctx.h, C.byref(os_), _p(p_ref), _p(p), C.byref(e)),
            "pam_darcy_error")
    return float(e.value)


# ---------------------------------------------------------------- learned warm start
CNN_PATCH = 16


def cnn_param_count() -> int:
    return int(N.lib().pam_cnn_param_count())


def _f32_dev(t: torch.Tensor, name: str) -> torch.Tensor:
    _require_cuda(t, name)
    if t.dtype != torch.float32:
        raise N.PamError(f"{name} must be float32")
    return t.contiguous()


def _patch_count(t: torch.Tensor, per: int, name: str) -> int:
    if t.numel() % per:
        raise N.PamError(f"{name} must hold whole 16x16 patches")
    return t.numel() // per


def _cnn_prec(precision: str) -> int:
    if precision not in ("f32", "bf16"):
        raise N.PamError("network precision must be 'f32' or 'bf16'")
    return N.PREC[precision]


def cnn_forward(ctx: Context, params: torch.Tensor, x: torch.Tensor,
                precision: str = "f32") -> torch.Tensor:
    """Logits [B, 2, 16, 16] of patches x [B, 1, 16, 16]; precision 'f32'
    (vector ALUs) or 'bf16' (32 -> 32 layers on MFMA)."""
    params, x = _f32_dev(params, "params"), _f32_dev(x, "x")
    B = _patch_count(x, 256, "x")
    out = torch.empty((B, 2, 16, 16), dtype=torch.float32, device=x.device)
    ctx.use_current_stream()
    N.check(N.lib().pam_cnn_forward(ctx.h, _p(params), B, _p(x), _p(out), _cnn_prec(precision)),
            "pam_cnn_forward")
    return out


def cnn_loss_grad(ctx: Context, params: torch.Tensor, x: torch.Tensor, target: torch.Tensor,
                  mask: torch.Tensor, grads: Optional[torch.Tensor] = None,
                  loss: Optional[torch.Tensor] = None, precision: str = "f32"):
    """(grads [P], loss scalar tensor) of the masked BCE over a batch."""
    params, x = _f32_dev(params, "params"), _f32_dev(x, "x")
    target, mask = _f32_dev(target, "target"), _f32_dev(mask, "mask")
    B = _patch_count(x, 256, "x")
    if _patch_count(target, 512, "target") != B or _patch_count(mask, 512, "mask") != B:
        raise N.PamError("target / mask must be [B, 2, 16, 16]")
    if grads is None:
        grads = torch.empty_like(params)
    if loss is None:
        loss = torch.empty((), dtype=torch.float32, device=x.device)
    ctx.use_current_stream()
    N.check(N.lib().pam_cnn_loss_grad(ctx.h, _p(params), B, _p(x), _p(target), _p(mask),
                                      _p(grads), _p(loss), _cnn_prec(precision)),
            "pam_cnn_loss_grad")
    return grads, loss


def cnn_adam(ctx: Context, params, grads, m, v, step: int, lr: float = 1e-3, beta1: float = 0.9,
             beta2: float = 0.999, eps: float = 1e-8):
    """One Adam step in place on params, m, v."""
    for t, n in ((params, "params"), (grads, "grads"), (m, "m"), (v, "v")):
        _f32_dev(t, n)
        if not t.is_contiguous():
            raise N.PamError(f"{n} must be contiguous")
    ctx.use_current_stream()
    N.check(N.lib().pam_cnn_adam(ctx.h, _p(params), _p(grads), _p(m), _p(v), int(step), float(lr),
                                 float(beta1), float(beta2), float(eps)), "pam_cnn_adam")


def grid_patches(ctx: Context, grid, cell_y: Optional[torch.Tensor] = None,
                 scale: float = 1.0 / 3.0) -> torch.Tensor:
    """16x16 patches [n, 1, 16, 16] of every owned box (value = scale * y)."""
    dev = torch.device("cuda", ctx.device)
    if cell_y is None:
        cell_y = torch.as_tensor(np.ascontiguousarray(grid.y, np.float64), device=dev)
    _require_cuda(cell_y, "cell_y")
    g, brk = _grid_struct(grid)
    n = C.c_int32()
    N.check(N.lib().pam_grid_patches(ctx.h, C.byref(g), None, C.c_float(scale), C.byref(n), None),
            "pam_grid_patches")
    out = torch.empty((n.value, 1, 16, 16), dtype=torch.float32, device=dev)
    ctx.use_current_stream()
    N.check(N.lib().pam_grid_patches(ctx.h, C.byref(g), _p(cell_y), C.c_float(scale), C.byref(n),
                                     _p(out)), "pam_grid_patches")
    return out


def support_hint(ctx: Context, grid, D: Dictionary, logits: torch.Tensor,
                 threshold: float = 0.0) -> torch.Tensor:
    """uint8 [n_sub, m_cap] hint from the support logits of the grid's patches."""
    logits = _f32_dev(logits, "logits")
    g, brk = _grid_struct(grid)
    out = torch.empty((D.n_sub, D.m_cap), dtype=torch.uint8, device=logits.device)
    ds = D.struct()
    ctx.use_current_stream()
    N.check(N.lib().pam_support_hint(ctx.h, C.byref(g), C.byref(ds), _p(logits), float(threshold),
                                     _p(out)), "pam_support_hint")
    return out


def cnn_labels(ctx: Context, grid, S: Samples, D: Dictionary, beta: torch.Tensor,
               elem_level: torch.Tensor):
    """(target, mask) [n, 2, 16, 16] from a cold fit's beta and one round's marks."""
    g, brk = _grid_struct(grid)
    n = C.c_int32()
    N.check(N.lib().pam_grid_patches(ctx.h, C.byref(g), None, C.c_float(1.0), C.byref(n), None),
            "pam_grid_patches")
    t = torch.empty((n.value, 2, 16, 16), dtype=torch.float32, device=beta.device)
    m = torch.empty_like(t)
    ss, ds = S.struct(), D.struct()
    ctx.use_current_stream()
    N.check(N.lib().pam_cnn_labels(ctx.h, C.byref(g), C.byref(ss), C.byref(ds), _p(beta),
                                   _p(elem_level), _p(t), _p(m)), "pam_cnn_labels")
    return t, m


def cnn_init(seed: int, device) -> torch.Tensor:
    """He-normal FP32 parameters on the device (seeded, see synth.cnn_init)."""
    from .synth import cnn_init as _init
    dev = torch.device("cuda", device) if isinstance(device, int) else device
    return torch.as_tensor(_init(seed), device=dev)


def cnn_train(ctx: Context, params: torch.Tensor, x: torch.Tensor, target: torch.Tensor,
              mask: torch.Tensor, epochs: int, batch: int = 256, lr: float = 2e-3, seed: int = 0,
              state=None, precision: str = "f32"):
    """Adam on the masked BCE over shuffled minibatches; params updated in
    place. Returns (mean loss per epoch, optimizer state (m, v, step))."""
    n = x.shape[0]
    if state is None:
        state = [torch.zeros_like(params), torch.zeros_like(params), 0]
    m, v = state[0], state[1]
    grads = torch.empty_like(params)
    gen = torch.Generator().manual_seed(seed)
    losses = []
    for _ in range(epochs):
        perm = torch.randperm(n, generator=gen).to(x.device)
        acc = torch.zeros((), dtype=torch.float64, device=x.device)
        nb = 0
        for b0 in range(0, n, batch):
            idx = perm[b0:b0 + batch]
            _, loss = cnn_loss_grad(ctx, params, x.index_select(0, idx), target.index_select(0, idx),
                                    mask.index_select(0, idx), grads, precision=precision)
            state[2] += 1
            cnn_adam(ctx, params, grads, m, v, state[2], lr)
            acc += loss
            nb += 1
        losses.append(float(acc) / max(nb, 1))
    return losses, state
