"""Pins of the oracle's per-subdomain choice of the elastic-net parameters
(Sec. 2 after Eq. (elastic); Exp. 1.2): an alpha path (lambda1 = rho alpha,
lambda2 = (1 - rho) alpha) scored by K-fold cross-validation.

Fixed independently of the oracle's code:
  - alpha_max is the zero threshold of the full-data fit: just above it the
    elastic net is exactly zero, just below it is not (KKT at beta = 0);
  - the grid is geometric from alpha_max to alpha_max * ratio;
  - every score equals the held-out squared error of fits found by
    enumerating all 3^M sign patterns (tiny M), on a Gaussian design
    normalized by its row sums written out here with numpy;
  - zero data give zero scores and the largest alpha (ties go to it);
  - the printed pair 4.59e-4 / 4.64e-6 is alpha = 4.64e-4 at rho = 0.99.
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_16564_amd import synth


def _one_subdomain(x, y, c, sigma):
    x = np.atleast_2d(np.asarray(x, float))
    if x.shape[0] == 1 and len(y) > 1:
        x = x.T
    N, d = x.shape
    M = len(sigma)
    D = O.Dictionary(1, M, d)
    D.m[0] = M
    D.c[:] = np.asarray(c, float).ravel()
    D.sigma[:] = sigma
    S = dict(off=np.array([0, N], np.int64), x=x, y=np.asarray(y, float))
    return S, D


def _design(x, c, sigma):
    """Row-normalized Gaussian design, written out directly."""
    x = np.asarray(x, float).reshape(len(x), -1)
    c = np.asarray(c, float).reshape(len(sigma), -1)
    r2 = ((x[:, None, :] - c[None, :, :]) ** 2).sum(-1)
    P = np.exp(-r2 / (2.0 * np.asarray(sigma)[None, :] ** 2))
    return P / P.sum(1, keepdims=True)


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


def test_printed_pair_is_alpha_at_mixing_099():
    a = 4.64e-4
    assert abs(0.99 * a - 4.59e-4) / 4.59e-4 < 1e-3 and abs(0.01 * a - 4.64e-6) / 4.64e-6 < 1e-12


def test_alpha_max_is_the_zero_threshold():
    g = synth.circle64(n=32, n_sub=2)
    S = O.partition(g)
    D = O.init_dictionary(g, [4, 4], 16)
    rho = 0.99
    alpha, score, best, l1, l2 = O.select_lambda(S, D, n_alpha=3, ratio=1e-2, rho=rho, k_folds=4)
    for s in range(D.n_sub):
        j0, j1 = S["off"][s], S["off"][s + 1]
        x, y = S["x"][j0:j1], S["y"][j0:j1]
        c = D.c[s * 16 * 2:(s + 1) * 16 * 2].reshape(16, 2)
        sg = D.sigma[s * 16:(s + 1) * 16]
        W = _design(x, c, sg)
        amax = np.abs(W.T @ y).max() / rho
        assert abs(alpha[s, 0] - amax) <= 1e-12 * amax
        if amax == 0.0:
            continue
        above = O.fit_one(x, y, c, sg, rho * amax * (1 + 1e-9), (1 - rho) * amax * (1 + 1e-9))[0]
        below = O.fit_one(x, y, c, sg, rho * amax * 0.999, (1 - rho) * amax * 0.999)[0]
        assert np.all(above == 0.0)
        assert np.any(below != 0.0)


def test_grid_is_geometric():
    g = synth.circle64(n=32, n_sub=2)
    S = O.partition(g)
    D = O.init_dictionary(g, [3, 3], 9)
    alpha, *_ = O.select_lambda(S, D, n_alpha=6, ratio=1e-3, k_folds=3)
    for s in range(D.n_sub):
        if alpha[s, 0] == 0.0:
            continue
        q = alpha[s, 1:] / alpha[s, :-1]
        assert np.allclose(q, (1e-3) ** (1 / 5), rtol=1e-12)
        assert abs(alpha[s, -1] / alpha[s, 0] - 1e-3) <= 1e-12


@pytest.mark.parametrize("seed", range(3))
def test_scores_match_brute_force_cross_validation(seed):
    rng = np.random.default_rng(400 + seed)
    N, M, K, n_alpha, rho = 14, 4, 3, 5, 0.9
    x = np.sort(rng.random(N))
    y = np.where(x < 0.45, -1.0, 2.0) + 0.1 * rng.normal(size=N)
    c = (np.arange(M) + 0.5) / M
    sg = np.full(M, 0.6 / M)
    S, D = _one_subdomain(x, y, c, sg)
    alpha, score, best, l1, l2 = O.select_lambda(S, D, n_alpha=n_alpha, ratio=1e-2, rho=rho,
                                                 k_folds=K)
    W = _design(x[:, None], c[:, None], sg)
    amax = np.abs(W.T @ y).max() / rho
    want = np.zeros(n_alpha)
    for k in range(n_alpha):
        a = amax * (1e-2) ** (k / (n_alpha - 1))
        assert abs(alpha[0, k] - a) <= 1e-12 * a
        err = 0.0
        for f in range(K):
            tr = np.arange(N) % K != f
            Wt = _design(x[tr, None], c[:, None], sg)
            beta = _brute_force(Wt.T @ Wt, Wt.T @ y[tr], rho * a, (1 - rho) * a)
            Wv = _design(x[~tr, None], c[:, None], sg)
            err += ((y[~tr] - Wv @ beta) ** 2).sum()
        want[k] = err / N
    assert np.allclose(score[0], want, rtol=1e-9, atol=1e-14)
    assert best[0] == int(np.argmin(want))
    assert l1[0] == rho * alpha[0, best[0]] and l2[0] == (1 - rho) * alpha[0, best[0]]


def test_zero_data_choose_the_largest_alpha():
    g = synth.circle64(n=32, n_sub=2)
    g.y = np.zeros_like(g.y)
    S = O.partition(g)
    D = O.init_dictionary(g, [3, 3], 9)
    alpha, score, best, l1, l2 = O.select_lambda(S, D, n_alpha=4, k_folds=3)
    assert np.all(score == 0.0) and np.all(best == 0) and np.all(alpha == 0.0)
