"""FP64 CPU oracle of the Darcy consumer of the reconstruction (Sec. 5, Eq.
(darcy_model) and the pressure experiment of Exp. 1: -div(K grad p) = 0 on a
box, p = 1 on the left face, p = 0 on the right face, no flow across the
others; continuous P1 finite elements; the relative L2 pressure error of
Eq. (pressure_L2_error)).

TEST INFRASTRUCTURE ONLY: imported by the test suite, never by the product
library. Plain numpy / scipy in float64, written from the definitions:

* mesh: n0 x n1 squares of the box, each split along its diagonal from
  vertex (i, j) to (i+1, j+1) into the lower-right triangle
  (i, j), (i+1, j), (i+1, j+1) and the upper-left triangle
  (i, j), (i+1, j+1), (i, j+1); nodes numbered i + (n0 + 1) j;
* K constant on each triangle (the caller evaluates it, e.g. at the
  centroid), array k_tri[j][i][t], t = 0 lower-right, 1 upper-left;
* stiffness: element by element, K |T| grad(phi_a) . grad(phi_b) with the
  barycentric gradients of each triangle (generic formula, no use of the
  structured shape), scattered into a sparse matrix;
* Dirichlet rows replaced by identity rows, their columns moved to the
  right-hand side (symmetric elimination); one sparse direct solve;
* norm: the L2(Omega) norm of a P1 function, by the exact P1 mass matrix.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def triangles(n0, n1):
    """Vertex indices [n1, n0, 2, 3] of every triangle."""
    j, i = np.meshgrid(np.arange(n1), np.arange(n0), indexing="ij")
    v00 = i + (n0 + 1) * j
    v10 = v00 + 1
    v01 = v00 + (n0 + 1)
    v11 = v01 + 1
    lr = np.stack([v00, v10, v11], -1)
    ul = np.stack([v00, v11, v01], -1)
    return np.stack([lr, ul], 2)


def nodes(n0, n1, lo, hi):
    xs = lo[0] + (hi[0] - lo[0]) * np.arange(n0 + 1) / n0
    ys = lo[1] + (hi[1] - lo[1]) * np.arange(n1 + 1) / n1
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    return np.column_stack([X.ravel(), Y.ravel()])


def centroids(n0, n1, lo, hi):
    """Triangle centroids [n1, n0, 2, 2]."""
    P = nodes(n0, n1, lo, hi)
    T = triangles(n0, n1)
    return P[T].mean(axis=-2)


def _local(P):
    """|T| and the barycentric gradients (3 x 2) of a triangle."""
    d1, d2 = P[1] - P[0], P[2] - P[0]
    det = d1[0] * d2[1] - d1[1] * d2[0]
    inv = np.array([[d2[1], -d2[0]], [-d1[1], d1[0]]]) / det
    g = np.vstack([-inv[0] - inv[1], inv[0], inv[1]])
    return abs(det) / 2.0, g


def stiffness(n0, n1, lo, hi, k_tri):
    P = nodes(n0, n1, lo, hi)
    T = triangles(n0, n1).reshape(-1, 3)
    K = np.asarray(k_tri, float).reshape(-1)
    rows, cols, vals = [], [], []
    for e in range(len(T)):
        area, g = _local(P[T[e]])
        Ae = K[e] * area * (g @ g.T)
        for a in range(3):
            for b in range(3):
                rows.append(T[e, a])
                cols.append(T[e, b])
                vals.append(Ae[a, b])
    n = (n0 + 1) * (n1 + 1)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def mass(n0, n1, lo, hi):
    P = nodes(n0, n1, lo, hi)
    T = triangles(n0, n1).reshape(-1, 3)
    rows, cols, vals = [], [], []
    for e in range(len(T)):
        area, _ = _local(P[T[e]])
        for a in range(3):
            for b in range(3):
                rows.append(T[e, a])
                cols.append(T[e, b])
                vals.append(area * (2.0 if a == b else 1.0) / 12.0)
    n = (n0 + 1) * (n1 + 1)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def solve(n0, n1, lo, hi, k_tri, p_left=1.0, p_right=0.0):
    """Nodal pressure [(n1+1)*(n0+1)], axis 0 fastest."""
    A = stiffness(n0, n1, lo, hi, k_tri).tolil()
    n = (n0 + 1) * (n1 + 1)
    i = np.arange(n) % (n0 + 1)
    dir_val = np.full(n, np.nan)
    dir_val[i == 0] = p_left
    dir_val[i == n0] = p_right
    is_d = ~np.isnan(dir_val)
    A = A.tocsr()
    pd = np.where(is_d, dir_val, 0.0)
    b = -A @ pd
    keep = ~is_d
    Aff = A[keep][:, keep]
    p = pd.copy()
    p[keep] = spla.spsolve(Aff.tocsc(), b[keep])
    return p


def l2_norm(n0, n1, lo, hi, u):
    M = mass(n0, n1, lo, hi)
    return float(np.sqrt(u @ (M @ u)))


def relative_error(n0, n1, lo, hi, p, p_star):
    """E_p = ||p - p*|| / ||p|| in L2(Omega) (Eq. (pressure_L2_error))."""
    return l2_norm(n0, n1, lo, hi, p - p_star) / l2_norm(n0, n1, lo, hi, p)


def k_from_cells(n0, n1, lo, hi, cell_y, c0, c1):
    """Permeability 10^y of the data cell (c0 x c1 cells on the same box)
    containing each triangle centroid: the true coefficient of the data."""
    C = centroids(n0, n1, lo, hi)
    ci = np.clip(np.floor((C[..., 0] - lo[0]) / (hi[0] - lo[0]) * c0).astype(int), 0, c0 - 1)
    cj = np.clip(np.floor((C[..., 1] - lo[1]) / (hi[1] - lo[1]) * c1).astype(int), 0, c1 - 1)
    return 10.0 ** np.asarray(cell_y).reshape(c1, c0)[cj, ci]
