"""Pins of the FP64 oracle of the learned warm start against things fixed
independently of it: a library correlation, central differences of the
loss, closed forms of the loss and of Adam, and structural identities of the
patch cut and of the hint / label maps."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import cnn_oracle as CO
from paper_2605_16564_amd import synth


def test_parameter_count():
    # 4 layers of 5x5 convolutions 1-32-32-32-2 with biases
    assert CO.param_count() == 53698
    assert synth.cnn_init(0).size == 53698


def test_conv_matches_library_correlation():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 16, 16))
    w = rng.standard_normal((4, 3, 5, 5))
    b = rng.standard_normal(4)
    out = CO.conv_same(x, w, b)
    for bi in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate2d(x[bi, c], w[o, c], mode="same", boundary="fill") for c in range(3))
            np.testing.assert_allclose(out[bi, o], ref, rtol=1e-13, atol=1e-12)


def _problem(seed, B=2):
    rng = np.random.default_rng(seed)
    p = synth.cnn_init(seed).astype(np.float64)
    p += 0.05 * rng.standard_normal(p.size)          # nonzero biases too
    x = rng.standard_normal((B, 1, 16, 16))
    t = (rng.random((B, 2, 16, 16)) < 0.4).astype(np.float64)
    m = (rng.random((B, 2, 16, 16)) < 0.7).astype(np.float64)
    return p, x, t, m


def test_gradient_matches_central_differences():
    p, x, t, m = _problem(3)
    _, g = CO.loss_grad(p, x, t, m)
    rng = np.random.default_rng(4)
    # indices in every layer's weights and biases
    idx = []
    o = 0
    for ci, co in zip(CO.CIN, CO.COUT):
        nw = co * ci * 25
        idx += list(o + rng.choice(nw, 6, replace=False)) + list(o + nw + rng.choice(co, 2, replace=False))
        o += nw + co
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (CO.loss_grad(pp, x, t, m)[0] - CO.loss_grad(pm, x, t, m)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3), (i, fd, g[i])


def test_bce_closed_forms():
    z = np.zeros((1, 2, 16, 16))
    t = np.random.default_rng(0).random(z.shape)
    loss, dz = CO.bce(z, t, np.ones_like(z))
    assert loss == pytest.approx(np.log(2.0), rel=1e-15)
    np.testing.assert_allclose(dz, (0.5 - t) / z.size, rtol=1e-15)
    # large positive logit with target 1: loss ~ exp(-z)
    zz = np.full((1, 2, 16, 16), 30.0)
    loss, _ = CO.bce(zz, np.ones_like(zz), np.ones_like(zz))
    assert loss == pytest.approx(np.exp(-30.0), rel=1e-12)
    # masked entries do not count; an empty mask gives zero
    m = np.zeros_like(z)
    m[0, 0, 3, 4] = 1.0
    z2 = z.copy()
    z2[0, 1] = 7.0
    assert CO.bce(z2, t, m)[0] == pytest.approx(CO.bce(z, t, m)[0], rel=1e-15)
    assert CO.bce(z, t, np.zeros_like(z))[0] == 0.0


def test_adam_constant_gradient_closed_form():
    # with a constant gradient the bias-corrected moments are g and g^2 at
    # every step, so each step moves lr * g / (|g| + eps)
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p0 = np.array([1.0, 2.0, 3.0, 4.0])
    p, m, v = p0.copy(), np.zeros(4), np.zeros(4)
    lr, eps = 0.01, 1e-8
    for step in range(1, 26):
        p, m, v = CO.adam(p, g, m, v, step, lr, eps=eps)
    np.testing.assert_allclose(p, p0 - 25 * lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)


def test_adam_minimizes_a_quadratic():
    p, m, v = np.array([0.0]), np.zeros(1), np.zeros(1)
    for step in range(1, 3001):
        p, m, v = CO.adam(p, p - 3.0, m, v, step, 0.05)
    assert abs(p[0] - 3.0) < 1e-3


def test_patches_tile_back_to_the_grid():
    grid = synth.facies256(seed=2001, n=64, n_sub=2)       # 2x2 subdomains of 32x32 cells
    scale = np.float32(1.0 / 3.0)
    pt = CO.patches(grid, scale)
    assert pt.shape == (16, 16, 16)
    Y = np.zeros((64, 64), np.float32)
    base, _ = CO.patch_index(grid)
    for s, (i0, j0, ni, nj) in enumerate(CO.owned_boxes_cells(grid)):
        for q in range((ni // 16) * (nj // 16)):
            pi, pj = q % (ni // 16), q // (ni // 16)
            Y[j0 + 16 * pj:j0 + 16 * pj + 16, i0 + 16 * pi:i0 + 16 * pi + 16] = pt[base[s] + q]
    ref = (np.float64(scale) * grid.y.reshape(64, 64)).astype(np.float32)
    assert np.array_equal(Y, ref)


def _cell_center_dictionary(grid, m_cap):
    """One center at the center of every owned cell (axis 0 fastest)."""
    boxes = CO.owned_boxes_cells(grid)
    h = 1.0 / grid.n_cells[0]
    c = np.zeros((len(boxes), m_cap, 2))
    m = np.zeros(len(boxes), np.int32)
    for s, (i0, j0, ni, nj) in enumerate(boxes):
        k = 0
        for j in range(nj):
            for i in range(ni):
                c[s, k] = ((i0 + i + 0.5) * h, (j0 + j + 0.5) * h)
                k += 1
        m[s] = k
    return m, c


def test_hint_reads_the_cell_of_each_center():
    grid = synth.facies256(seed=2001, n=64, n_sub=2)
    m_cap = 32 * 32 + 5
    m, c = _cell_center_dictionary(grid, m_cap)
    _, tot = CO.patch_index(grid)
    P = 16
    # logit of pixel (r, q) of patch p: +1 if (p + r + 2q) % 3 == 0 else -1
    lg = np.zeros((tot, 2, P, P), np.float32)
    for p in range(tot):
        for r in range(P):
            for q in range(P):
                lg[p, 1, r, q] = 1.0 if (p + r + 2 * q) % 3 == 0 else -1.0
    hn = CO.hint(grid, m, c, m_cap, lg, 0.0)
    base, _ = CO.patch_index(grid)
    for s, (i0, j0, ni, nj) in enumerate(CO.owned_boxes_cells(grid)):
        for k in range(m[s]):
            i, j = k % ni, k // ni                               # owned cell of center k
            p = base[s] + (j // P) * (ni // P) + i // P
            assert hn[s, k] == (1 if (p + j % P + 2 * (i % P)) % 3 == 0 else 0)
        assert not hn[s, m[s]:].any()


def test_labels_from_beta_and_marks():
    grid = synth.facies256(seed=2001, n=64, n_sub=2)
    m_cap = 32 * 32
    m, c = _cell_center_dictionary(grid, m_cap)
    n_sub = 4
    beta = np.zeros((n_sub, m_cap))
    beta[:, ::3] = 0.5                                          # every third center active
    # samples: the cell centers of every owned box (no overlap), same order
    off = np.arange(n_sub + 1) * 1024
    x = c.reshape(-1, 2)
    lvl = (np.arange(n_sub * 1024) % 5 == 0).astype(np.int32)    # every fifth element marked
    t, mk = CO.labels(grid, off, x, m, c, m_cap, beta, lvl)
    base, _ = CO.patch_index(grid)
    assert mk.sum() == 2 * 64 * 64                              # every cell labelled in both channels
    for s, (i0, j0, ni, nj) in enumerate(CO.owned_boxes_cells(grid)):
        for k in range(m[s]):
            i, j = k % ni, k // ni
            p = base[s] + (j // 16) * (ni // 16) + i // 16
            assert t[p, 1, j % 16, i % 16] == (1.0 if k % 3 == 0 else 0.0)
            assert t[p, 0, j % 16, i % 16] == (1.0 if (s * 1024 + k) % 5 == 0 else 0.0)


def test_bf16_rounding_closed_forms():
    # 8-bit significand: spacing 2^-7 on [1, 2); round to nearest, ties to even
    cases = [(1.0, 1.0), (1.0 + 2.0 ** -9, 1.0), (1.0 + 2.0 ** -8, 1.0),      # below half, tie -> even
             (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),                           # tie -> even (up)
             (1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + 2.0 ** -7),                  # above half
             (-3.0 - 2.0 ** -7, -3.0), (0.0, 0.0), (2.0 ** -130, 2.0 ** -130)]  # subnormal kept
    for x, want in cases:
        assert CO.bf16(np.array([x]))[0] == want, (x, CO.bf16(np.array([x]))[0], want)


def test_bf16_emulation_only_touches_listed_layers():
    p, x, t, m = _problem(5)
    z0, _ = CO.forward(p, x)
    z1, _ = CO.forward(p, x, bf16_layers=(1, 2))
    rel = np.abs(z1 - z0).max() / np.abs(z0).max()
    assert 0.0 < rel < 5e-2          # a rounding-size change
    # rounding nothing reproduces the plain network exactly
    assert np.array_equal(CO.forward(p, x, bf16_layers=())[0], z0)

