"""Pins of the Darcy consumer oracle (Sec. 5 Eq. (darcy_model), the pressure
experiment of Exp. 1, Eq. (pressure_L2_error)), from what the mathematics
fixes:
  - constant K, or K varying only across the flow (layers parallel to it):
    the exact pressure p = p_left + (p_right - p_left) x is linear and lies
    in the P1 space, so the discrete solution equals it;
  - K varying only along the flow (layers in series): the flux is the same
    through every column, so the nodal pressure drops by h_i / K_i per
    column (closed form);
  - the stiffness on these right triangles is an M-matrix: the discrete
    maximum principle keeps p in [p_right, p_left] for any positive K;
  - the flux entering on the left equals the flux leaving on the right;
  - the mass-matrix norm integrates P1 functions exactly (1 and x);
  - mirror symmetry of K across the mid-line mirrors p.
"""
import numpy as np
import pytest

from oracle import darcy_oracle as DO


def _grid(n0=12, n1=9, lo=(0.5, -1.0), hi=(2.0, 1.0)):
    return n0, n1, np.array(lo, float), np.array(hi, float)


def test_constant_and_cross_layers_give_the_linear_pressure():
    n0, n1, lo, hi = _grid()
    X = DO.nodes(n0, n1, lo, hi)
    lin = 1.0 - (X[:, 0] - lo[0]) / (hi[0] - lo[0])
    p = DO.solve(n0, n1, lo, hi, np.full((n1, n0, 2), 3.7))
    assert np.abs(p - lin).max() <= 1e-12
    rng = np.random.default_rng(1)
    layers = 10.0 ** rng.uniform(-2, 2, size=n1)
    k = np.broadcast_to(layers[:, None, None], (n1, n0, 2)).copy()
    p = DO.solve(n0, n1, lo, hi, k)
    assert np.abs(p - lin).max() <= 1e-10


def test_series_layers_closed_form():
    n0, n1, lo, hi = _grid()
    rng = np.random.default_rng(2)
    kc = 10.0 ** rng.uniform(-2, 2, size=n0)
    k = np.broadcast_to(kc[None, :, None], (n1, n0, 2)).copy()
    p = DO.solve(n0, n1, lo, hi, k, p_left=2.0, p_right=-1.0)
    h = (hi[0] - lo[0]) / n0
    drop = np.concatenate([[0.0], np.cumsum(h / kc)])
    want = 2.0 - 3.0 * drop / drop[-1]
    P = p.reshape(n1 + 1, n0 + 1)
    assert np.abs(P - want[None, :]).max() <= 1e-10


def test_maximum_principle_and_flux_balance():
    n0, n1, lo, hi = _grid(16, 14)
    rng = np.random.default_rng(3)
    k = 10.0 ** rng.uniform(-3, 3, size=(n1, n0, 2))
    p = DO.solve(n0, n1, lo, hi, k)
    assert p.min() >= -1e-12 and p.max() <= 1.0 + 1e-12
    A = DO.stiffness(n0, n1, lo, hi, k)
    react = A @ p                       # zero at free nodes, boundary fluxes at Dirichlet nodes
    i = np.arange(len(p)) % (n0 + 1)
    free = (i > 0) & (i < n0)
    assert np.abs(react[free]).max() <= 1e-9 * np.abs(react).max()
    q_in, q_out = react[i == 0].sum(), react[i == n0].sum()
    assert q_in > 0 and abs(q_in + q_out) <= 1e-9 * q_in


def test_mass_norm_is_exact_on_p1_functions():
    n0, n1, lo, hi = _grid()
    X = DO.nodes(n0, n1, lo, hi)
    area = np.prod(hi - lo)
    assert abs(DO.l2_norm(n0, n1, lo, hi, np.ones(len(X))) - np.sqrt(area)) <= 1e-12
    want = (hi[0] ** 3 - lo[0] ** 3) / 3.0 * (hi[1] - lo[1])
    assert abs(DO.l2_norm(n0, n1, lo, hi, X[:, 0]) ** 2 - want) <= 1e-12 * want
    assert DO.relative_error(n0, n1, lo, hi, X[:, 0] + 1, X[:, 0] + 1) == 0.0


def test_mirror_symmetry():
    n0, n1, lo, hi = _grid(10, 8, (0.0, 0.0), (1.0, 1.0))
    rng = np.random.default_rng(4)
    cell = 10.0 ** rng.uniform(-2, 2, size=(n1, n0))
    k = np.repeat(cell[:, :, None], 2, axis=2)           # one value per square
    km = np.repeat(cell[::-1, :, None], 2, axis=2)       # mirrored across y = 1/2
    p = DO.solve(n0, n1, lo, hi, k).reshape(n1 + 1, n0 + 1)
    pm = DO.solve(n0, n1, lo, hi, km).reshape(n1 + 1, n0 + 1)
    # the diagonal split is not mirror-symmetric, but with one value per
    # square the edge couplings are, so the nodal solution mirrors
    assert np.abs(p - pm[::-1]).max() <= 1e-10


def test_k_from_cells_reads_the_containing_cell():
    n0, n1, lo, hi = 8, 6, np.array([0.0, 0.0]), np.array([1.0, 1.0])
    y = np.arange(4 * 3, dtype=float).reshape(3, 4)    # 4 x 3 data cells
    k = DO.k_from_cells(n0, n1, lo, hi, y.ravel(), 4, 3)
    assert k.shape == (n1, n0, 2)
    assert k[0, 0, 0] == 1.0 and k[5, 7, 1] == 10.0 ** 11
    assert np.all(k[:, 0:2, :] == 10.0 ** y[np.arange(n1) // 2, 0][:, None, None])
