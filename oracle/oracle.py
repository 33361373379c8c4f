"""ctypes binding of the FP64 CPU oracle (oracle/pam_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product library. It builds the
plain C file with gcc (no HIP, no shared code with the library).

Each wrapper names the step of the paper it mirrors; the C file cites the
sections in detail.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "pam_oracle.c"
_LIB = _HERE / "_build" / "libpam_oracle.so"

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_lp = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def build(force: bool = False) -> Path:
    """Compile the oracle with gcc: FP64, no FMA contraction, OpenMP over subdomains."""
    _LIB.parent.mkdir(parents=True, exist_ok=True)
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp")
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
            "-fno-fast-math", "-fopenmp", "-o", str(tmp), str(_SRC), "-lm",
        ])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(str(build()))
        L.ora_partition_count.restype = C.c_long
        L.ora_partition_count.argtypes = [C.c_int, _ip, _ip, _ip, C.c_double, _lp]
        L.ora_partition_gather.restype = C.c_int
        L.ora_partition_gather.argtypes = [C.c_int, _ip, _dp, _dp, _ip, _ip, C.c_double,
                                           _dp, _lp, _dp, _dp, _dp, _ip]
        L.ora_lattice.restype = C.c_int
        L.ora_lattice.argtypes = [C.c_int, _dp, _dp, _ip, C.c_double, _dp, _dp, _ip]
        L.ora_design.restype = C.c_int
        L.ora_design.argtypes = [C.c_int, C.c_int, C.c_int, _dp, _dp, _dp, _dp]
        L.ora_normal.restype = None
        L.ora_normal.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp, _dp]
        L.ora_cd.restype = C.c_int
        L.ora_cd.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_double, C.c_int, C.c_double, _dp]
        L.ora_fss.restype = C.c_int
        L.ora_fss.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_double, C.c_int, C.c_double, _dp]
        L.ora_kkt.restype = C.c_double
        L.ora_kkt.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_double, _dp]
        L.ora_fit_one.restype = C.c_int
        L.ora_fit_one.argtypes = [C.c_int, C.c_int, C.c_int, _dp, _dp, _dp, _dp, C.c_double,
                                  C.c_double, C.c_int, _dp, _dp]
        L.ora_indicator.restype = None
        L.ora_indicator.argtypes = [C.c_int, C.c_int, C.c_int, _dp, _dp, _dp, _dp, _dp, _dp,
                                    C.c_int, _dp]
        L.ora_mark.restype = C.c_int
        L.ora_mark.argtypes = [C.c_int, _dp, C.c_int, C.c_double, _ip]
        L.ora_enrich.restype = C.c_int
        L.ora_enrich.argtypes = [C.c_int, C.c_int, C.c_int, _dp, _dp, C.c_int, _ip, C.c_double,
                                 C.c_double, _ip, _dp, _dp, _ip]
        L.ora_fit_batch.restype = C.c_int
        L.ora_fit_batch.argtypes = [C.c_int, C.c_int, _lp, _dp, _dp, C.c_int, _ip, _dp, _dp,
                                    C.c_double, C.c_double, C.c_int, _dp, _dp, _ip]
        L.ora_refine_batch.restype = C.c_int
        L.ora_refine_batch.argtypes = [C.c_int, C.c_int, _lp, _dp, _dp, _dp, C.c_int, _ip, _dp,
                                       _dp, _ip, _dp, _ip, C.c_double, C.c_double, C.c_int,
                                       _ip, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int,
                                       _dp, _ip, _ip]
        L.ora_eval.restype = C.c_long
        L.ora_eval.argtypes = [C.c_int, _ip, _dp, C.c_int, _ip, _dp, _dp, _dp, C.c_long, _dp,
                               C.c_int, _dp]
        L.ora_eval_blend.restype = C.c_long
        L.ora_eval_blend.argtypes = [C.c_int, _ip, _dp, C.c_double, C.c_int, _ip, _dp, _dp, _dp,
                                     C.c_long, _dp, C.c_int, _dp]
        L.ora_interface_jump.restype = C.c_long
        L.ora_interface_jump.argtypes = [C.c_int, _ip, _dp, C.c_int, _ip, _dp, _dp, _dp, C.c_int,
                                         _dp]
        L.ora_select_lambda.restype = C.c_int
        L.ora_select_lambda.argtypes = [C.c_int, C.c_int, _lp, _dp, _dp, C.c_int, _ip, _dp, _dp,
                                        C.c_int, C.c_double, C.c_double, C.c_int, C.c_int, _dp,
                                        _dp, _ip]
        L.ora_set_basis.restype = None
        L.ora_set_basis.argtypes = [C.c_int]
        _lib = L
    return _lib


def _basis(basis):
    """Select the basis for the next oracle call ("shepard": the normalized
    functions of Sec. 3.2; "plain": the unnormalized Gaussians of Example 1)."""
    if basis not in ("shepard", "plain"):
        raise ValueError("basis must be 'shepard' or 'plain'")
    lib().ora_set_basis(1 if basis == "plain" else 0)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# ---------------------------------------------------------------- a1 / a2
def partition(grid) -> dict:
    """Samples of every subdomain of a structured grid (Sec. 2 Steps 1-2).

    `grid` is a `paper_2605_16564_amd.synth.Grid`-like object with fields
    dim, n_cells, lo, hi, n_sub, breaks (list of per-axis cell-index
    breakpoints), overlap, y (cell values, axis 0 fastest)."""
    d = grid.dim
    nc = _i32(grid.n_cells[:d])
    ns = _i32(grid.n_sub[:d])
    brk = _i32(np.concatenate([np.asarray(b) for b in grid.breaks[:d]]))
    n_tot = int(np.prod(ns))
    off = np.zeros(n_tot + 1, np.int64)
    total = lib().ora_partition_count(d, nc, ns, brk, float(grid.overlap), off)
    if total < 0:
        raise ValueError("bad partition arguments")
    x = np.zeros(total * d)
    y = np.zeros(total)
    h = np.zeros(total * d)
    cell = np.zeros(total * d, np.int32)
    st = lib().ora_partition_gather(d, nc, _f64(grid.lo[:d]), _f64(grid.hi[:d]), ns, brk,
                                    float(grid.overlap), _f64(grid.y.ravel()), off, x, y, h, cell)
    if st != 0:
        raise RuntimeError("partition gather failed")
    return dict(off=off, x=x.reshape(total, d), y=y, h=h.reshape(total, d),
                cell=cell.reshape(total, d))


def lattice(box_lo, box_hi, g, sigma_factor=1.0):
    """Initial g^d lattice dictionary of one owned box (Exp. 1 setup)."""
    d = len(g)
    M = int(np.prod(g))
    c = np.zeros(M * d)
    s = np.zeros(M)
    lv = np.zeros(M, np.int32)
    lib().ora_lattice(d, _f64(box_lo), _f64(box_hi), _i32(g), float(sigma_factor), c, s, lv)
    return c.reshape(M, d), s, lv


# ---------------------------------------------------------------- a3-a6
def design(x, c, sigma, basis="shepard"):
    x = _f64(x); c = _f64(c)
    _basis(basis)
    N, d = x.shape
    M = c.shape[0]
    W = np.zeros((N, M))
    st = lib().ora_design(d, N, M, x.ravel(), c.ravel(), _f64(sigma), W.reshape(-1))
    if st != 0:
        raise FloatingPointError("Shepard denominator underflow")
    return W


def normal(W, y):
    W = _f64(W)
    N, M = W.shape
    G = np.zeros((M, M))
    b = np.zeros(M)
    lib().ora_normal(N, M, W.reshape(-1), _f64(y), G.reshape(-1), b)
    return G, b


def cd(G, b, lambda1, lambda2, sweeps, beta=None, tol=1e-13):
    M = len(b)
    beta = np.zeros(M) if beta is None else _f64(beta).copy()
    n = lib().ora_cd(M, _f64(G).reshape(-1), _f64(b), lambda1, lambda2, sweeps, tol, beta)
    return beta, n


def fss(G, b, lambda1, lambda2, beta=None, max_iter=100000, kkt_tol=1e-12):
    M = len(b)
    beta = np.zeros(M) if beta is None else _f64(beta).copy()
    it = lib().ora_fss(M, _f64(G).reshape(-1), _f64(b), lambda1, lambda2, max_iter, kkt_tol, beta)
    return beta, it


def kkt(G, b, lambda1, lambda2, beta):
    return lib().ora_kkt(len(b), _f64(G).reshape(-1), _f64(b), lambda1, lambda2, _f64(beta))


def fit_one(x, y, c, sigma, lambda1, lambda2, cd_sweeps=8, beta=None, basis="shepard"):
    """Steps a3-a6 on one subdomain; returns (beta, status, stats)."""
    x = _f64(x); c = _f64(c)
    _basis(basis)
    N, d = x.shape
    M = c.shape[0]
    beta = np.zeros(M) if beta is None else _f64(beta).copy()
    stats = np.zeros(3)
    st = lib().ora_fit_one(d, N, M, x.ravel(), _f64(y), c.ravel(), _f64(sigma), lambda1, lambda2,
                           cd_sweeps, beta, stats)
    return beta, st, stats


def indicator(x, y, h, c, sigma, beta, space=0, basis="shepard"):
    x = _f64(x); c = _f64(c)
    _basis(basis)
    N, d = x.shape
    R = np.zeros(N)
    lib().ora_indicator(d, N, c.shape[0], x.ravel(), _f64(y), _f64(h).ravel(), c.ravel(),
                        _f64(sigma), _f64(beta), space, R)
    return R


def mark(R, k_top, tol):
    R = _f64(R)
    out = np.zeros(max(k_top, 1), np.int32)
    n = lib().ora_mark(len(R), R, k_top, tol, out)
    return out[:n]


# ---------------------------------------------------------------- batched
class Dictionary:
    """Capacity-padded per-subdomain dictionary (same layout as the library's)."""

    def __init__(self, n_sub, m_cap, dim):
        self.n_sub, self.m_cap, self.dim = n_sub, m_cap, dim
        self.m = np.zeros(n_sub, np.int32)
        self.c = np.zeros(n_sub * m_cap * dim)
        self.sigma = np.zeros(n_sub * m_cap)
        self.level = np.zeros(n_sub * m_cap, np.int32)
        self.basis = "shepard"

    def copy(self):
        o = Dictionary(self.n_sub, self.m_cap, self.dim)
        o.m = self.m.copy(); o.c = self.c.copy(); o.sigma = self.sigma.copy()
        o.level = self.level.copy()
        o.basis = self.basis
        return o


def init_dictionary(grid, g, m_cap, sigma_factor=1.0, basis="shepard") -> Dictionary:
    """Lattice dictionary for every owned box of a grid partition (a2)."""
    d = grid.dim
    boxes = grid_owned_boxes(grid)
    D = Dictionary(len(boxes), m_cap, d)
    D.basis = basis
    M = int(np.prod(g[:d]))
    for s, (lo, hi) in enumerate(boxes):
        c, sg, lv = lattice(lo, hi, list(g[:d]), sigma_factor)
        D.m[s] = M
        D.c[s * m_cap * d:(s * m_cap + M) * d] = c.ravel()
        D.sigma[s * m_cap:s * m_cap + M] = sg
        D.level[s * m_cap:s * m_cap + M] = lv
    return D


def grid_axis_coords(grid):
    """Owned breakpoints per axis in coordinates: lo + b * h_cell."""
    out = []
    for a in range(grid.dim):
        hcell = (grid.hi[a] - grid.lo[a]) / grid.n_cells[a]
        out.append(np.array([grid.lo[a] + float(b) * hcell for b in grid.breaks[a]]))
    return out


def grid_owned_boxes(grid):
    ax = grid_axis_coords(grid)
    d = grid.dim
    ns = list(grid.n_sub[:d]) + [1] * (3 - d)
    boxes = []
    for k2 in range(ns[2]):
        for k1 in range(ns[1]):
            for k0 in range(ns[0]):
                kk = (k0, k1, k2)
                lo = np.array([ax[a][kk[a]] for a in range(d)])
                hi = np.array([ax[a][kk[a] + 1] for a in range(d)])
                boxes.append((lo, hi))
    return boxes


def fit_batch(samples, D: Dictionary, lambda1, lambda2, cd_sweeps=8, beta=None):
    d = D.dim
    n = D.n_sub
    beta = np.zeros(n * D.m_cap) if beta is None else _f64(beta).copy()
    stats = np.zeros(3 * n)
    status = np.zeros(n, np.int32)
    _basis(D.basis)
    lib().ora_fit_batch(d, n, samples["off"], _f64(samples["x"]).ravel(), _f64(samples["y"]),
                        D.m_cap, D.m, D.c, D.sigma, lambda1, lambda2, cd_sweeps, beta, stats,
                        status)
    return beta, status, stats.reshape(n, 3)


def refine_batch(samples, D: Dictionary, lambda1, lambda2, k_top, max_rounds, m_max, eps_tol,
                 eta=0.5, space=0, cd_sweeps=8, beta=None, elem_level=None):
    """Alg. 1 on every subdomain. Mutates a copy of D; returns (D, beta, elem_level, info)."""
    D = D.copy()
    d = D.dim
    n = D.n_sub
    N_tot = len(samples["y"])
    beta = np.zeros(n * D.m_cap) if beta is None else _f64(beta).copy()
    lvl = np.zeros(N_tot, np.int32) if elem_level is None else _i32(elem_level).copy()
    k_top = _i32(np.broadcast_to(np.asarray(k_top, np.int32), (n,)))
    rs = np.zeros(n * (max_rounds + 1) * 5)
    rounds = np.zeros(n, np.int32)
    status = np.zeros(n, np.int32)
    _basis(D.basis)
    lib().ora_refine_batch(d, n, samples["off"], _f64(samples["x"]).ravel(),
                           _f64(samples["y"]), _f64(samples["h"]).ravel(), D.m_cap, D.m, D.c,
                           D.sigma, D.level, beta, lvl, lambda1, lambda2, cd_sweeps, k_top,
                           max_rounds, m_max, eps_tol, eta, space, rs, rounds, status)
    info = dict(round_stats=rs.reshape(n, max_rounds + 1, 5), rounds=rounds, status=status)
    return D, beta, lvl, info


def evaluate(axis_x, D: Dictionary, beta, xq, space=0):
    """Global reconstruction K*(x) at query points (Sec. 2 Step 4)."""
    d = D.dim
    xq = _f64(xq).reshape(-1, d)
    Q = xq.shape[0]
    out = np.zeros(Q)
    ns = _i32([len(a) - 1 for a in axis_x])
    ax = _f64(np.concatenate(axis_x))
    _basis(D.basis)
    n_out = lib().ora_eval(d, ns, ax, D.m_cap, D.m, D.c, D.sigma, _f64(beta), Q, xq.ravel(),
                           space, out)
    return out, n_out


def evaluate_blend(axis_x, D: Dictionary, beta, xq, blend, space=0):
    """Continuous reconstruction: partition-of-unity average of neighbouring
    local surrogates (Sec. 2 Step 4 and the remark after it); the weights are
    defined in the C file. blend = 0 is the owner reconstruction."""
    d = D.dim
    xq = _f64(xq).reshape(-1, d)
    Q = xq.shape[0]
    out = np.zeros(Q)
    ns = _i32([len(a) - 1 for a in axis_x])
    ax = _f64(np.concatenate(axis_x))
    _basis(D.basis)
    n_out = lib().ora_eval_blend(d, ns, ax, float(blend), D.m_cap, D.m, D.c, D.sigma, _f64(beta),
                                 Q, xq.ravel(), space, out)
    return out, n_out


def interface_count(n_sub):
    """Interior interface pieces of a box partition with n_sub per axis."""
    n_sub = list(n_sub)
    tot = int(np.prod(n_sub))
    return sum(tot // n_sub[a] * (n_sub[a] - 1) for a in range(len(n_sub)))


def interface_jump(axis_x, D: Dictionary, beta, n):
    """Per interior interface piece (axis, then the upper subdomain in linear
    order): (max, mean) of |K*_A - K*_B| at n^(dim-1) face midpoints."""
    d = D.dim
    ns = _i32([len(a) - 1 for a in axis_x])
    nf = interface_count(ns)
    out = np.zeros(2 * max(nf, 1))
    ax = _f64(np.concatenate(axis_x))
    _basis(D.basis)
    got = lib().ora_interface_jump(d, ns, ax, D.m_cap, D.m, D.c, D.sigma, _f64(beta), int(n), out)
    assert got == nf
    return out[:2 * nf].reshape(nf, 2)


def select_lambda(samples, D: Dictionary, n_alpha=8, ratio=1e-3, rho=0.99, k_folds=5, cd_sweeps=8):
    """Per-subdomain elastic-net strength by a path over alpha = lambda1 +
    lambda2 (lambda1 = rho alpha) and K-fold cross-validation; the reading is
    stated in the C file. Returns (alpha [n_sub, n_alpha], score [n_sub,
    n_alpha], best [n_sub], lambda1 [n_sub], lambda2 [n_sub])."""
    n = D.n_sub
    alpha = np.zeros(n * n_alpha)
    score = np.zeros(n * n_alpha)
    best = np.zeros(n, np.int32)
    _basis(D.basis)
    bad = lib().ora_select_lambda(D.dim, n, samples["off"], _f64(samples["x"]).ravel(),
                                  _f64(samples["y"]), D.m_cap, D.m, D.c, D.sigma, int(n_alpha),
                                  float(ratio), float(rho), int(k_folds), int(cd_sweeps), alpha,
                                  score, best)
    if bad:
        raise RuntimeError(f"{bad} oracle fits failed")
    alpha, score = alpha.reshape(n, n_alpha), score.reshape(n, n_alpha)
    a = alpha[np.arange(n), best]
    return alpha, score, best, rho * a, (1.0 - rho) * a
