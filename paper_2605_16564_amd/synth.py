"""Seeded synthetic inputs for the PAM hot path.

This module produces inputs only: cellwise-constant log10 coefficient fields on
structured grids, subdomain breakpoints, query points and the quadrature points
of the error metrics. It contains none of the method's arithmetic (no basis
functions, normalization, regression, indicator or enrichment), so both the
HIP library and the CPU oracle can consume what it generates.

Workloads (the paper's own Case 1/2 fields and the SPE10 data are not
available; these synthetic stand-ins reproduce their sizes and structure):

* ``circle64``   2-D 64x64 unit square, log10 K = 3 inside the circle of
  radius 0.3 at (0.5, 0.5), 0 outside; 2x2 subdomains with 10 % overlap,
  16x16 centers per subdomain, FP64, plain fit.
* ``facies256``  2-D 256x256 three-facies field: Gaussian random field with
  squared-exponential covariance (correlation length 0.05) thresholded at its
  33rd/66th percentiles into log10 K in {-1, 1, 3}; 8x8 subdomains, 12x12
  initial centers, up to 3 refinement rounds.
* ``layered3d``  3-D 60x220x85 layered field alternating smooth log-normal
  layers and channelized layers; 6x22x9 subdomains, 8x8x8 centers.
* ``multifield`` 64 independent 2-D disc-facies fields of sizes 64^2..512^2,
  each with 10^6 uniform query points.

All randomness uses numpy's PCG64 with fixed seeds.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# Elastic-net parameters printed for the 1-D study (Sec. 3.5, Example 2);
# used as the default for every workload.
LAMBDA1 = 4.59e-4
LAMBDA2 = 4.64e-6


@dataclass
class Grid:
    """Structured grid with cellwise values and a box partition.

    y holds log10 K per cell with axis 0 fastest (C order of shape
    (n_cells[2], n_cells[1], n_cells[0]) flattened)."""

    dim: int
    n_cells: List[int]
    lo: List[float]
    hi: List[float]
    n_sub: List[int]
    breaks: List[np.ndarray]
    overlap: float
    y: np.ndarray

    @property
    def n_subdomains(self) -> int:
        return int(np.prod(self.n_sub[: self.dim]))

    @property
    def cell_size(self) -> np.ndarray:
        return np.array([(self.hi[a] - self.lo[a]) / self.n_cells[a] for a in range(self.dim)])


def even_breaks(n: int, k: int) -> np.ndarray:
    """Cell-index breakpoints floor(i*n/k), i = 0..k."""
    return np.array([(i * n) // k for i in range(k + 1)], dtype=np.int32)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def cell_centers_2d(n0: int, n1: int, lo=(0.0, 0.0), hi=(1.0, 1.0)):
    x = lo[0] + (np.arange(n0) + 0.5) * (hi[0] - lo[0]) / n0
    yv = lo[1] + (np.arange(n1) + 0.5) * (hi[1] - lo[1]) / n1
    X, Y = np.meshgrid(x, yv, indexing="xy")  # shape (n1, n0): axis 0 fastest
    return X, Y


def grf_2d(n: int, corr_len_cells: float, rng: np.random.Generator, pad: int = 2) -> np.ndarray:
    """Unit-variance Gaussian random field with covariance exp(-r^2/(2 l^2)) by
    FFT spectral synthesis on a periodic (pad*n)^2 grid, cropped to n x n."""
    m = pad * n
    k = np.fft.fftfreq(m)  # cycles per cell
    KX, KY = np.meshgrid(k, k, indexing="ij")
    spec = np.exp(-2.0 * np.pi ** 2 * corr_len_cells ** 2 * (KX ** 2 + KY ** 2))
    white = rng.standard_normal((m, m))
    z = np.real(np.fft.ifft2(np.fft.fft2(white) * np.sqrt(spec)))[:n, :n]
    z = (z - z.mean()) / z.std()
    return z


# ----------------------------------------------------------------- workloads
def circle64(n: int = 64, n_sub: int = 2, overlap: float = 0.1) -> Grid:
    X, Y = cell_centers_2d(n, n)
    y = np.where((X - 0.5) ** 2 + (Y - 0.5) ** 2 < 0.09, 3.0, 0.0)
    return Grid(2, [n, n, 1], [0.0, 0.0, 0.0], [1.0, 1.0, 1.0], [n_sub, n_sub, 1],
                [even_breaks(n, n_sub), even_breaks(n, n_sub), even_breaks(1, 1)],
                overlap, y.ravel().astype(np.float64))


def facies256(seed: int = 2000, n: int = 256, n_sub: int = 8) -> Grid:
    rng = _rng(seed)
    z = grf_2d(n, 0.05 * n, rng)
    flat = np.sort(z.ravel())
    t1 = flat[int(np.floor(0.33 * flat.size))]
    t2 = flat[int(np.floor(0.66 * flat.size))]
    y = np.where(z < t1, -1.0, np.where(z < t2, 1.0, 3.0))
    return Grid(2, [n, n, 1], [0.0, 0.0, 0.0], [1.0, 1.0, 1.0], [n_sub, n_sub, 1],
                [even_breaks(n, n_sub), even_breaks(n, n_sub), even_breaks(1, 1)],
                0.0, y.ravel().astype(np.float64))


def facies_mosaic(seed: int, tiles: int = 8) -> Grid:
    """tiles x tiles independent facies256 fields (seeds seed, seed+1, ...)
    side by side: the same cells (1/256), subdomains (32 x 32 cells) and
    facies statistics as facies256, on [0, tiles]^2."""
    n = 256 * tiles
    Y = np.zeros((n, n))
    for tj in range(tiles):
        for ti in range(tiles):
            f = facies256(seed=seed + tj * tiles + ti)
            Y[tj * 256:(tj + 1) * 256, ti * 256:(ti + 1) * 256] = f.y.reshape(256, 256)
    return Grid(2, [n, n, 1], [0.0, 0.0, 0.0], [float(tiles), float(tiles), 1.0], [8 * tiles, 8 * tiles, 1],
                [even_breaks(n, 8 * tiles), even_breaks(n, 8 * tiles), even_breaks(1, 1)], 0.0, Y.ravel())


def layered3d(nx: int = 60, ny: int = 220, nz: int = 85, sub=(6, 22, 9), seed: int = 3000) -> Grid:
    """Layered 3-D field: even layers 1 + 1.5 z with z a unit-variance GRF
    (correlation length 10 cells); odd layers a constant background in
    U(-2, 0) cut by 2-4 sinusoidal channels along axis 1 (width 3-8 cells,
    value U(3, 4))."""
    y = np.zeros((nz, ny, nx))
    X, Y = np.meshgrid(np.arange(nx) + 0.5, np.arange(ny) + 0.5, indexing="xy")  # (ny, nx)
    for k in range(nz):
        rng = _rng(seed + k)
        if k % 2 == 0:
            z = grf_2d(max(nx, ny), 10.0, rng)[:ny, :nx]
            y[k] = 1.0 + 1.5 * z
        else:
            layer = np.full((ny, nx), rng.uniform(-2.0, 0.0))
            for _ in range(int(rng.integers(2, 5))):
                x0 = rng.uniform(0.0, nx)
                amp = rng.uniform(2.0, 8.0)
                lam = rng.uniform(40.0, 120.0)
                ph = rng.uniform(0.0, 2.0 * np.pi)
                width = int(rng.integers(3, 9))
                val = rng.uniform(3.0, 4.0)
                centre = x0 + amp * np.sin(2.0 * np.pi * Y / lam + ph)
                layer = np.where(np.abs(X - centre) < 0.5 * width, val, layer)
            y[k] = layer
    return Grid(3, [nx, ny, nz], [0.0, 0.0, 0.0], [float(nx), float(ny), float(nz)],
                list(sub), [even_breaks(nx, sub[0]), even_breaks(ny, sub[1]),
                            even_breaks(nz, sub[2])], 0.0, y.ravel().astype(np.float64))


def disc_field(seed: int, n: Optional[int] = None, cells_per_sub: int = 32,
               overlap: float = 0.1) -> Grid:
    """One multi-field member: side n = 32 * U{2..16}, F ~ U{2..5} facies with
    levels linspace(0, 3, F); background level 0 and F-1 discs (centers
    U(0.2, 0.8)^2, radii U(0.1, 0.3)) painted in order with levels 1..F-1."""
    rng = _rng(seed)
    if n is None:
        n = 32 * int(rng.integers(2, 17))
    F = int(rng.integers(2, 6))
    levels = np.linspace(0.0, 3.0, F)
    X, Y = cell_centers_2d(n, n)
    y = np.full((n, n), levels[0])
    for f in range(1, F):
        cx, cy = rng.uniform(0.2, 0.8, size=2)
        r = rng.uniform(0.1, 0.3)
        y = np.where((X - cx) ** 2 + (Y - cy) ** 2 < r * r, levels[f], y)
    ns = n // cells_per_sub
    return Grid(2, [n, n, 1], [0.0, 0.0, 0.0], [1.0, 1.0, 1.0], [ns, ns, 1],
                [even_breaks(n, ns), even_breaks(n, ns), even_breaks(1, 1)], overlap,
                y.ravel().astype(np.float64))


def multifield(n_fields: int = 64, seed0: int = 5000) -> List[Grid]:
    return [disc_field(seed0 + f) for f in range(n_fields)]


def uniform_queries(dim: int, Q: int, seed: int, lo=None, hi=None, dtype=np.float32) -> np.ndarray:
    lo = np.zeros(dim) if lo is None else np.asarray(lo[:dim], np.float64)
    hi = np.ones(dim) if hi is None else np.asarray(hi[:dim], np.float64)
    u = _rng(seed).random((Q, dim))
    return (lo + u * (hi - lo)).astype(dtype)


# ----------------------------------------------------------------- 1-D and small fixtures
def step1d(n_cells: int = 64) -> Grid:
    """Example 1 step: Omega = [0, 0.03125], jump at 0.015625 from 1e-4 to
    1e-1 (log10 -4 to -1); the paper does not give the sample count."""
    L = 0.03125
    xc = (np.arange(n_cells) + 0.5) * L / n_cells
    y = np.where(xc < 0.015625, -4.0, -1.0)
    return Grid(1, [n_cells, 1, 1], [0.0, 0.0, 0.0], [L, 1.0, 1.0], [1, 1, 1],
                [even_breaks(n_cells, 1), even_breaks(1, 1), even_breaks(1, 1)], 0.0,
                y.astype(np.float64))


# Three-Gaussian partition-of-unity example of Sec. 3.2.
PU_CENTERS = np.array([[0.3, 0.3], [0.7, 0.4], [0.5, 0.75]])
PU_SIGMAS = np.array([0.10, 0.15, 0.07])


def random_points(dim: int, n: int, seed: int, lo=0.0, hi=1.0) -> np.ndarray:
    return lo + (hi - lo) * _rng(seed).random((n, dim))


# ----------------------------------------------------------------- error metric points
def gauss_legendre(n: int):
    x, w = np.polynomial.legendre.leggauss(n)
    return x, w


def metric_points(grid: Grid, n_per_axis: int, cells: Optional[np.ndarray] = None):
    """Tensor Gauss-Legendre points inside cells (all cells, or the listed flat
    cell indices). Returns (points [P, d], weights [P], flat cell index [P])."""
    d = grid.dim
    nc = grid.n_cells[:d]
    h = grid.cell_size
    if cells is None:
        cells = np.arange(int(np.prod(nc)))
    cells = np.asarray(cells, np.int64)
    idx = []
    rem = cells.copy()
    for a in range(d):
        idx.append(rem % nc[a])
        rem //= nc[a]
    gx, gw = gauss_legendre(n_per_axis)
    grids = np.meshgrid(*([np.arange(n_per_axis)] * d), indexing="ij")
    combos = np.stack([g.ravel() for g in grids], 1)  # [n^d, d]
    P = len(cells) * len(combos)
    pts = np.zeros((len(cells), len(combos), d))
    wts = np.ones((len(cells), len(combos)))
    for a in range(d):
        centre = grid.lo[a] + (idx[a] + 0.5) * h[a]
        pts[:, :, a] = centre[:, None] + 0.5 * h[a] * gx[combos[:, a]][None, :]
        wts *= 0.5 * h[a] * gw[combos[:, a]][None, :]
    cell_of = np.repeat(cells, len(combos))
    return pts.reshape(P, d), wts.reshape(P), cell_of


# ----------------------------------------------------------------- workload parameters
@dataclass
class Workload:
    name: str
    grids: List[Grid]
    g: List[int]                 # initial lattice per axis
    sigma_factor: float = 1.0    # sigma0 = factor * max_axis(h_c)
    lambda1: float = LAMBDA1
    lambda2: float = LAMBDA2
    precision: str = "f64"      # Gram precision: f64 | f32 | bf16
    k_top: int = 0               # 0: no refinement
    k_top_frac: float = 0.0      # alternative: floor(frac * N_i)
    max_rounds: int = 0
    eta: float = 0.5
    eps_tol_rel: float = 1e-4    # eps_tol = rel * |T|
    queries_per_field: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def m0(self) -> int:
        return int(np.prod(self.g[: self.grids[0].dim]))


def workload(name: str) -> Workload:
    if name == "circle64":
        return Workload(name, [circle64()], [16, 16], precision="f64")
    if name == "facies256":
        return Workload(name, [facies256()], [12, 12], precision="f32", k_top=204,
                        max_rounds=3)
    if name == "layered3d":
        return Workload(name, [layered3d()], [8, 8, 8], precision="f32", k_top_frac=0.05,
                        max_rounds=3)
    if name == "multifield":
        return Workload(name, multifield(), [16, 16], precision="f32",
                        queries_per_field=1_000_000)
    raise KeyError(name)


# ---------------------------------------------------------------- network inputs
CNN_LAYERS = ((1, 32), (32, 32), (32, 32), (32, 2))   # (cin, cout) of the 5x5 layers
CNN_SCALE = 1.0 / 3.0                                   # patch value = y / 3


def cnn_init(seed: int) -> np.ndarray:
    """He-normal weights (std sqrt(2 / (cin * 25))) and zero biases, float32,
    per layer w[cout][cin][5][5] then b[cout]."""
    rng = _rng(seed)
    parts = []
    for ci, co in CNN_LAYERS:
        parts.append(rng.standard_normal(co * ci * 25) * np.sqrt(2.0 / (ci * 25)))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


def cnn_batch(seed: int, B: int, p_target: float = 0.4, p_mask: float = 0.7):
    """Random patches [B,1,16,16] (three-level values / 3 with noise), binary
    targets and masks [B,2,16,16], float32."""
    rng = _rng(seed)
    x = (rng.integers(-1, 2, (B, 1, 16, 16)) * 2 + 1) / 3.0 + 0.05 * rng.standard_normal((B, 1, 16, 16))
    t = (rng.random((B, 2, 16, 16)) < p_target).astype(np.float32)
    m = (rng.random((B, 2, 16, 16)) < p_mask).astype(np.float32)
    return x.astype(np.float32), t, m


def random_coefficients(seed: int, n_sub: int, m_cap: int, m) -> np.ndarray:
    """Coefficients [n_sub, m_cap] of field-like size (normal, std 2) with
    about a quarter exactly zero; slots >= m[s] are zero."""
    rng = _rng(seed)
    b = 2.0 * rng.standard_normal((n_sub, m_cap))
    b[rng.random((n_sub, m_cap)) < 0.25] = 0.0
    for s in range(n_sub):
        b[s, int(m[s]):] = 0.0
    return b

