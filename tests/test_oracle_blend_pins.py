"""Pins of the oracle's interface treatment (Sec. 2 Step 4 and the remark
after it): the partition-of-unity average of neighbouring local surrogates
and the jump of the piecewise reconstruction across interfaces.

What fixes the answers here, independently of the oracle's formulas:
  - local surrogates that are constants (every coefficient of subdomain i
    equal to c_i makes the Shepard expansion exactly c_i) turn the blend
    into the weighted mean of the c_i: all equal gives that constant at
    every point (partition of unity); on an interface the symmetric ramp
    gives the midpoint of the two constants, at a corner the mean of the
    2^d constants; across a band the value runs monotonically from one
    constant to the other;
  - blend 0 and points outside every band reduce to the owner
    reconstruction, which the older pins already fix;
  - the blended field is continuous and C1 (finite differences), while
    the owner reconstruction jumps by exactly the interface jump (limits
    from both sides);
  - constant surrogates give interface jumps |c_A - c_B| with the faces in
    the documented order.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_16564_amd.synth import Grid

pytestmark = pytest.mark.filterwarnings("ignore")


def _grid2():
    # uneven 3 x 2 partition of a 30 x 20 grid on [0, 3] x [1, 3]
    return Grid(2, [30, 20, 1], [0.0, 1.0, 0.0], [3.0, 3.0, 1.0], [3, 2, 1],
                [np.array([0, 8, 18, 30], np.int32), np.array([0, 12, 20], np.int32),
                 np.array([0, 1], np.int32)], 0.0, np.zeros(600))


def _grid3():
    return Grid(3, [6, 6, 6], [0.0, 0.0, 0.0], [1.0, 1.0, 1.0], [2, 2, 2],
                [np.array([0, 3, 6], np.int32), np.array([0, 2, 6], np.int32),
                 np.array([0, 4, 6], np.int32)], 0.0, np.zeros(216))


def _dict(g, lat, cap, seed):
    D = O.init_dictionary(g, lat, cap)
    rng = np.random.default_rng(seed)
    beta = rng.standard_normal(D.n_sub * cap)
    return D, beta


def _const_beta(D, consts):
    beta = np.zeros(D.n_sub * D.m_cap)
    for s in range(D.n_sub):
        beta[s * D.m_cap:(s + 1) * D.m_cap] = consts[s]
    return beta


def _random_points(g, Q, seed):
    rng = np.random.default_rng(seed)
    lo, hi = np.array(g.lo[:g.dim]), np.array(g.hi[:g.dim])
    return lo + rng.random((Q, g.dim)) * (hi - lo)


@pytest.mark.parametrize("grid", [_grid2, _grid3])
@pytest.mark.parametrize("blend", [0.05, 0.25, 0.5])
def test_equal_constants_are_reproduced(grid, blend):
    g = grid()
    D, _ = _dict(g, [3] * g.dim, 27, 1)
    beta = _const_beta(D, np.full(D.n_sub, 1.75))
    x = _random_points(g, 4000, 2)
    v, n_out = O.evaluate_blend(O.grid_axis_coords(g), D, beta, x, blend)
    assert n_out == 0
    assert np.abs(v - 1.75).max() <= 1e-14


@pytest.mark.parametrize("blend", [0.1, 0.3])
def test_interface_midpoints_and_corners_2d(blend):
    g = _grid2()
    ax = O.grid_axis_coords(g)
    D, _ = _dict(g, [3, 3], 9, 3)
    consts = np.array([0.0, 1.0, 4.0, 9.0, 16.0, 25.0])   # subdomain (k0, k1) -> k0 + 3 k1
    beta = _const_beta(D, consts)
    # on the axis-0 breakpoint between (0,0) and (1,0), away from the axis-1 band
    pts = [[ax[0][1], 1.2], [ax[0][2], 2.9], [1.3, ax[1][1]], [ax[0][1], ax[1][1]],
           [ax[0][2], ax[1][1]]]
    v, _ = O.evaluate_blend(ax, D, beta, np.array(pts), blend)
    want = [(0 + 1) / 2, (16 + 25) / 2, (1 + 16) / 2, (0 + 1 + 9 + 16) / 4, (1 + 4 + 16 + 25) / 4]
    assert np.abs(v - want).max() <= 1e-14 * consts.max()


def test_corner_3d_is_the_mean_of_eight():
    g = _grid3()
    ax = O.grid_axis_coords(g)
    D, _ = _dict(g, [2, 2, 2], 8, 4)
    consts = np.arange(8, dtype=np.float64) ** 2
    v, _ = O.evaluate_blend(ax, D, _const_beta(D, consts),
                            np.array([[ax[0][1], ax[1][1], ax[2][1]]]), 0.2)
    assert abs(v[0] - consts.mean()) <= 1e-14 * consts.max()


def test_transition_is_monotone_between_the_constants():
    g = _grid2()
    ax = O.grid_axis_coords(g)
    D, _ = _dict(g, [3, 3], 9, 5)
    consts = np.array([-1.0, 2.0, 0.0, 0.0, 0.0, 0.0])
    beta = _const_beta(D, consts)
    blend = 0.25
    L0, L1 = ax[0][1] - ax[0][0], ax[0][2] - ax[0][1]
    h = blend * min(L0, L1)
    t = np.linspace(ax[0][1] - 1.5 * h, ax[0][1] + 1.5 * h, 301)
    x = np.column_stack([t, np.full_like(t, 1.3)])
    v, _ = O.evaluate_blend(ax, D, beta, x, blend)
    assert np.all(np.diff(v) >= -1e-15)
    assert np.all(v[t <= ax[0][1] - h] == -1.0) and np.all(v[t >= ax[0][1] + h] == 2.0)
    assert np.all((v >= -1.0) & (v <= 2.0))


@pytest.mark.parametrize("grid", [_grid2, _grid3])
def test_blend_zero_is_the_owner_reconstruction(grid):
    g = grid()
    ax = O.grid_axis_coords(g)
    D, beta = _dict(g, [3] * g.dim, 27, 6)
    x = _random_points(g, 3000, 7)
    # exact breakpoints and domain faces exercise the half-open rule
    x[:50, 0] = np.resize(ax[0], 50)
    x[50:100, 1] = np.resize(ax[1], 50)
    v, n0 = O.evaluate_blend(ax, D, beta, x, 0.0)
    o, n1 = O.evaluate(ax, D, beta, x)
    assert n0 == n1 == 0
    assert np.array_equal(v, o)


def test_points_outside_every_band_take_the_owner_value():
    g = _grid2()
    ax = O.grid_axis_coords(g)
    D, beta = _dict(g, [3, 3], 9, 8)
    blend = 0.1
    x = _random_points(g, 6000, 9)
    keep = np.ones(len(x), bool)
    for a in range(2):
        b = ax[a]
        for i in range(1, len(b) - 1):
            h = blend * min(b[i] - b[i - 1], b[i + 1] - b[i])
            keep &= np.abs(x[:, a] - b[i]) >= h
    assert keep.sum() > 1000 and (~keep).sum() > 500
    v, _ = O.evaluate_blend(ax, D, beta, x, blend)
    o, _ = O.evaluate(ax, D, beta, x)
    assert np.array_equal(v[keep], o[keep])
    assert not np.array_equal(v[~keep], o[~keep])


def test_blend_is_continuous_and_c1_where_the_owner_field_jumps():
    g = _grid2()
    ax = O.grid_axis_coords(g)
    D, beta = _dict(g, [4, 4], 16, 10)
    blend = 0.2
    b = ax[0][1]
    y = 1.7
    eps = 1e-9
    xs = np.array([[b - eps, y], [b + eps, y]])
    v, _ = O.evaluate_blend(ax, D, beta, xs, blend)
    o, _ = O.evaluate(ax, D, beta, xs)
    jump = abs(o[0] - o[1])
    assert jump > 1e-3            # the independent fits disagree at the interface
    assert abs(v[0] - v[1]) <= 1e-6
    # C1 at a band edge: one-sided slopes agree to O(step)
    h = blend * min(ax[0][1] - ax[0][0], ax[0][2] - ax[0][1])
    for e in (b - h, b + h):
        d = 1e-5
        f, _ = O.evaluate_blend(ax, D, beta, np.array([[e - d, y], [e, y], [e + d, y]]), blend)
        left, right = (f[1] - f[0]) / d, (f[2] - f[1]) / d
        assert abs(left - right) <= 1e-3 * max(1.0, abs(left))


def test_points_outside_the_domain_are_nan():
    g = _grid2()
    ax = O.grid_axis_coords(g)
    D, beta = _dict(g, [3, 3], 9, 11)
    x = np.array([[-0.01, 2.0], [1.0, 3.0001], [3.0, 3.0]])
    v, n_out = O.evaluate_blend(ax, D, beta, x, 0.3)
    assert n_out == 2 and np.isnan(v[0]) and np.isnan(v[1]) and np.isfinite(v[2])


def test_interface_jump_of_constants_in_face_order():
    g = _grid2()
    ax = O.grid_axis_coords(g)
    D, _ = _dict(g, [3, 3], 9, 12)
    consts = np.array([0.0, 1.0, 4.0, 9.0, 16.0, 25.0])
    J = O.interface_jump(ax, D, _const_beta(D, consts), 5)
    # axis 0: B = 1, 2, 4, 5 (A = B - 1); axis 1: B = 3, 4, 5 (A = B - 3)
    pairs = [(0, 1), (1, 2), (3, 4), (4, 5), (0, 3), (1, 4), (2, 5)]
    want = np.array([abs(consts[b] - consts[a]) for a, b in pairs])
    assert J.shape == (7, 2) == (O.interface_count([3, 2]), 2)
    tol = 1e-14 * consts.max()
    assert np.abs(J[:, 0] - want).max() <= tol and np.abs(J[:, 1] - want).max() <= tol


@pytest.mark.parametrize("grid", [_grid2, _grid3])
def test_interface_jump_is_the_limit_difference_of_the_owner_field(grid):
    g = grid()
    ax = O.grid_axis_coords(g)
    D, beta = _dict(g, [3] * g.dim, 27, 13)
    J = O.interface_jump(ax, D, beta, 1)   # one sample: the face midpoint
    ns = [len(a) - 1 for a in ax]
    stride = [1, ns[0], ns[0] * (ns[1] if g.dim > 1 else 1)]
    f = 0
    eps = 1e-9
    for a in range(g.dim):
        for B in range(int(np.prod(ns))):
            kk = [B % ns[0], (B // ns[0]) % (ns[1] if g.dim > 1 else 1),
                  B // (ns[0] * (ns[1] if g.dim > 1 else 1))]
            if kk[a] == 0:
                continue
            mid = np.array([0.5 * (ax[b][kk[b]] + ax[b][kk[b] + 1]) if b != a else ax[b][kk[b]]
                            for b in range(g.dim)])
            lo, hi = mid.copy(), mid.copy()
            lo[a] -= eps
            hi[a] += eps
            o, _ = O.evaluate(ax, D, beta, np.array([lo, hi]))
            assert abs(abs(o[0] - o[1]) - J[f, 0]) <= 1e-6
            assert J[f, 0] == J[f, 1]
            assert B - stride[a] >= 0
            f += 1
    assert f == len(J)
