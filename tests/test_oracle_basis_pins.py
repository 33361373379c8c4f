"""Pins of the oracle's plain (unnormalized) basis, the construction the paper
compares the Shepard-normalized one against in Example 1 (Sec. 3.2):

  - two Gaussians with unit coefficients: the plain expansion is
    phi_1 + phi_2, which exceeds 1 between close centers (the amplified
    overlap of Example 1), the normalized one is exactly 1;
  - the elastic-net fit on the plain design equals the unique KKT point
    found by enumerating every sign pattern on a design written out here;
  - the indicator of the plain expansion equals the Gauss-Legendre sum of
    its squared misfit computed here directly;
  - the switch does not leak: a Shepard call after a plain one gives the
    Shepard answer again;
  - the indicator on K itself (Alg. 1 literal, the other ablation) equals
    the Gauss-Legendre sum of the squared misfit of 10^K* against 10^y.
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as O


def _raw(x, c, sigma):
    x = np.asarray(x, float).reshape(len(x), -1)
    c = np.asarray(c, float).reshape(len(sigma), -1)
    r2 = ((x[:, None, :] - c[None, :, :]) ** 2).sum(-1)
    return np.exp(-r2 / (2.0 * np.asarray(sigma)[None, :] ** 2))


def _one(c, sigma, beta, basis):
    c = np.asarray(c, float).reshape(len(sigma), -1)
    D = O.Dictionary(1, len(sigma), c.shape[1])
    D.m[0] = len(sigma)
    D.c[:] = c.ravel()
    D.sigma[:] = sigma
    D.basis = basis
    ax = [np.array([-10.0, 10.0])] * c.shape[1]
    return D, ax


def test_two_gaussians_amplify_without_normalization():
    sigma = np.array([0.1, 0.1])
    for d in (0.05, 0.1, 0.2, 0.4):
        c = np.array([[0.0], [d]])
        mid = np.array([[d / 2]])
        Dp, ax = _one(c, sigma, None, "plain")
        vp, _ = O.evaluate(ax, Dp, np.ones(2), mid)
        Ds, _ = _one(c, sigma, None, "shepard")
        vs, _ = O.evaluate(ax, Ds, np.ones(2), mid)
        want = 2.0 * np.exp(-(d / 2) ** 2 / (2 * 0.1 ** 2))
        assert abs(vp[0] - want) <= 1e-15 * want
        assert abs(vs[0] - 1.0) <= 1e-15
        assert (vp[0] > 1.0) == (d < 0.1 * np.sqrt(8 * np.log(2)))


def _brute_force(G, b, l1, l2):
    M = len(b)
    A = G + l2 * np.eye(M)
    sols = []
    for th in itertools.product((-1.0, 0.0, 1.0), repeat=M):
        th = np.array(th)
        S = np.nonzero(th)[0]
        beta = np.zeros(M)
        if len(S):
            beta[S] = np.linalg.solve(A[np.ix_(S, S)], b[S] - l1 * th[S])
            if np.any(np.sign(beta[S]) != th[S]):
                continue
        g = b - A @ beta
        Z = np.nonzero(th == 0)[0]
        if len(Z) and np.max(np.abs(g[Z])) > l1 * (1 + 1e-10):
            continue
        sols.append(beta)
    assert len(sols) == 1
    return sols[0]


@pytest.mark.parametrize("seed", range(3))
def test_plain_fit_matches_brute_force(seed):
    rng = np.random.default_rng(600 + seed)
    x = rng.random((18, 2))
    c = rng.random((5, 2))
    sg = rng.uniform(0.15, 0.4, size=5)
    y = np.where(x[:, 0] + x[:, 1] > 1.0, 2.0, -1.0)
    Phi = _raw(x, c, sg)
    l1, l2 = 0.05, 1e-3
    want = _brute_force(Phi.T @ Phi, Phi.T @ y, l1, l2)
    W = O.design(x, c, sg, basis="plain")
    assert np.allclose(W, Phi, rtol=1e-15, atol=0)
    beta, st, _ = O.fit_one(x, y, c, sg, l1, l2, basis="plain")
    assert st == 0
    assert np.abs(beta - want).max() <= 1e-10 * max(1.0, np.abs(want).max())
    # and the Shepard fit of the same data is a different problem
    bs, _, _ = O.fit_one(x, y, c, sg, l1, l2)
    assert np.abs(bs - beta).max() > 1e-3


def test_plain_indicator_is_the_quadrature_of_the_misfit():
    rng = np.random.default_rng(610)
    x = rng.random((7, 2))
    h = np.full((7, 2), 0.1)
    y = rng.normal(size=7)
    c = rng.random((4, 2))
    sg = np.full(4, 0.3)
    beta = rng.normal(size=4)
    R = O.indicator(x, y, h, c, sg, beta, basis="plain")
    off = 0.1 / (2 * np.sqrt(3))
    want = np.zeros(7)
    for q in itertools.product((-1, 1), repeat=2):
        xq = x + off * np.array(q)
        want += 0.01 / 4 * (_raw(xq, c, sg) @ beta - y) ** 2
    assert np.allclose(R, want, rtol=1e-13, atol=0)


def test_switch_does_not_leak():
    x = np.array([[0.2, 0.3]])
    c = np.array([[0.0, 0.0], [0.5, 0.5]])
    sg = np.array([0.3, 0.3])
    w1 = O.design(x, c, sg)
    O.design(x, c, sg, basis="plain")
    w2 = O.design(x, c, sg)
    assert np.array_equal(w1, w2) and abs(w1.sum() - 1.0) <= 1e-15


def test_linear_space_indicator_is_the_quadrature_of_the_k_misfit():
    """Alg. 1 literal: R_T measured on K = 10^(log10 K) rather than on the
    log values (the ablation of the indicator space)."""
    rng = np.random.default_rng(611)
    x = rng.random((6, 2))
    h = np.full((6, 2), 0.2)
    y = rng.normal(size=6)
    c = rng.random((5, 2))
    sg = np.full(5, 0.25)
    beta = rng.normal(size=5)
    R = O.indicator(x, y, h, c, sg, beta, space=1)
    off = 0.2 / (2 * np.sqrt(3))
    want = np.zeros(6)
    for q in itertools.product((-1, 1), repeat=2):
        P = _raw(x + off * np.array(q), c, sg)
        v = (P @ beta) / P.sum(1)
        want += 0.04 / 4 * (10.0 ** v - 10.0 ** y) ** 2
    assert np.allclose(R, want, rtol=1e-12, atol=0)
