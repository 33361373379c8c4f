"""The oracle's elastic-net minimizer, certified without the oracle's own code.

Eq. (elastic) (solved exactly, Sec. 3.3) is
    P(beta) = 1/2 ||y - W beta||^2 + lambda1 ||beta||_1 + lambda2/2 ||beta||^2.
Written as a Lasso on augmented data, W^ = [W; sqrt(lambda2) I] and
y^ = [y; 0], its dual is D(theta) = 1/2 ||y^||^2 - 1/2 ||y^ - theta||^2 over
||W^' theta||_inf <= lambda1. For any beta, theta = s r^ with r^ = y^ - W^ beta
and s = min(1, lambda1 / ||W^' r^||_inf) is dual feasible, so
gap(beta) = P(beta) - D(theta) >= P(beta) - P* >= 0: a certificate of how far
beta is from optimal, computed here with numpy from a design written out
here (not the oracle's). P is strongly convex with modulus
mu = lambda_min(W'W) + lambda2, so ||beta - beta*||^2 <= 2 gap(beta) / mu.

Checks: the oracle's fits have a gap at rounding level, where a relative
change of 1e-3 in one coefficient (or beta = 0) gives a gap larger by many
orders of magnitude; an independent solver (scikit-learn's cyclic coordinate
descent, a different algorithm and code base) reaches the same support and
no lower objective, and the two solutions lie within the distance the two
gaps allow. Inputs: 32 x 32 cell patches of the seeded facies256 field,
lattice dictionaries and a dictionary with groups of three half-width centers
at random cells (the shape of an enriched one), Shepard and plain bases.
"""
import warnings

import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_16564_amd import synth

L1, L2 = synth.LAMBDA1, synth.LAMBDA2
H = 1.0 / 256


@pytest.fixture(scope="module")
def field():
    return np.asarray(synth.facies256().y, np.float64).reshape(256, 256)


def _patch(Y, i0, j0, n=32):
    xs = (np.arange(n) + 0.5) * H
    X1, X2 = np.meshgrid(i0 * H + xs, j0 * H + xs, indexing="xy")
    return np.stack([X1.ravel(), X2.ravel()], 1), Y[j0:j0 + n, i0:i0 + n].ravel().copy()


def _lattice(i0, j0, g, n=32):
    L = n * H
    cs = (np.arange(g) + 0.5) * L / g
    C1, C2 = np.meshgrid(i0 * H + cs, j0 * H + cs, indexing="xy")
    return np.stack([C1.ravel(), C2.ravel()], 1), np.full(g * g, L / g)


def _enriched(x, c, sig, n_groups, seed):
    """Add, at n_groups random sample points, the three centers offset by
    half a cell along each axis and both, with half the lattice width."""
    rng = np.random.default_rng(seed)
    pick = rng.choice(len(x), n_groups, replace=False)
    off = np.array([[0.5, 0.0], [0.0, 0.5], [0.5, 0.5]]) * H
    ex = (x[pick][:, None, :] + off[None, :, :]).reshape(-1, 2)
    return np.vstack([c, ex]), np.concatenate([sig, np.full(len(ex), 0.5 * sig[0])])


def _design(x, c, sig, plain):
    d2 = ((x[:, None, :] - c[None, :, :]) ** 2).sum(-1)
    P = np.exp(-d2 / (2.0 * sig[None, :] ** 2))
    return P if plain else P / P.sum(1, keepdims=True)


def _primal(W, y, b):
    r = y - W @ b
    return 0.5 * r @ r + L1 * np.abs(b).sum() + 0.5 * L2 * b @ b


def _gap(W, y, b):
    r = y - W @ b
    rb = -np.sqrt(L2) * b
    corr = W.T @ r + np.sqrt(L2) * rb
    s = min(1.0, L1 / np.abs(corr).max())
    t1, t2 = s * r, s * rb
    dual = 0.5 * y @ y - 0.5 * ((y - t1) @ (y - t1) + t2 @ t2)
    return _primal(W, y, b) - dual


def _certify(W, y, b):
    """The oracle's beta is optimal to rounding, and the certificate tells it
    apart from small perturbations."""
    yy = float(y @ y)
    g = _gap(W, y, b)
    bound = 1e-11 * yy
    assert -1e-9 <= g <= bound, (g, bound)
    k = int(np.argmax(np.abs(b)))
    bp = b.copy()
    bp[k] *= 1.001
    assert _gap(W, y, bp) > 1e3 * bound
    assert _gap(W, y, np.zeros_like(b)) > 1e3 * bound
    return g


@pytest.mark.parametrize("i0,j0,g", [(0, 0, 12), (96, 32, 12)])
def test_lattice_fit_certified_and_matches_coordinate_descent(field, i0, j0, g):
    from sklearn.linear_model import ElasticNet
    x, y = _patch(field, i0, j0)
    c, sig = _lattice(i0, j0, g)
    W = _design(x, c, sig, plain=False)
    b, st, _ = O.fit_one(x, y, c, sig, L1, L2)
    assert st == 0
    g_o = _certify(W, y, b)
    N = len(y)
    # the same objective divided by N: alpha * l1_ratio = lambda1 / N,
    # alpha * (1 - l1_ratio) = lambda2 / N
    en = ElasticNet(alpha=(L1 + L2) / N, l1_ratio=L1 / (L1 + L2), fit_intercept=False,
                    tol=1e-15, max_iter=200_000, precompute=True, selection="cyclic")
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        en.fit(W, y)
    bs = en.coef_
    assert np.array_equal(b != 0.0, bs != 0.0)
    p_o, p_s = _primal(W, y, b), _primal(W, y, bs)
    assert p_o <= p_s + 1e-13 * p_o
    g_s = max(_gap(W, y, bs), 0.0)
    mu = float(np.linalg.eigvalsh(W.T @ W)[0]) + L2
    dist = float(np.linalg.norm(b - bs))
    assert dist <= np.sqrt(2.0 * max(g_o, 0.0) / mu) + np.sqrt(2.0 * g_s / mu) + 1e-12, (dist, g_o, g_s, mu)


def test_enriched_dictionary_fit_certified(field):
    """744 centers of two widths on 1,024 samples (the size of a first
    refinement round): the gap certificate at a size where the brute-force
    sign enumeration cannot reach."""
    x, y = _patch(field, 64, 96)
    c, sig = _enriched(x, *_lattice(64, 96, 12), n_groups=200, seed=160)
    assert len(c) == 744
    W = _design(x, c, sig, plain=False)
    b, st, _ = O.fit_one(x, y, c, sig, L1, L2)
    assert st == 0
    _certify(W, y, b)
    assert 0 < np.count_nonzero(b) < len(c)


def test_plain_basis_fit_certified(field):
    x, y = _patch(field, 160, 200)
    c, sig = _lattice(160, 200, 12)
    W = _design(x, c, sig, plain=True)
    b, st, _ = O.fit_one(x, y, c, sig, L1, L2, basis="plain")
    assert st == 0
    _certify(W, y, b)


def test_duplicated_centers_share_the_coefficient(field):
    """Two identical columns make the Gram exactly singular; lambda2 > 0
    keeps the objective strictly convex, so the minimizer is unique and
    symmetric in the two copies: each gets the same coefficient (the
    elastic net's grouping of equal columns), and the gap certifies it."""
    x, y = _patch(field, 32, 64)
    c, sig = _lattice(32, 64, 8)
    dup = [0, 9, 30, 63]
    c2, s2 = np.vstack([c, c[dup]]), np.concatenate([sig, sig[dup]])
    W = _design(x, c2, s2, plain=False)
    b, st, _ = O.fit_one(x, y, c2, s2, L1, L2)
    assert st == 0
    _certify(W, y, b)
    scale = np.abs(b).max()
    for i, k in enumerate(dup):
        assert abs(b[64 + i] - b[k]) <= 1e-9 * scale, (k, b[64 + i], b[k])
