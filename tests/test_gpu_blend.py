"""GPU parity of the interface treatment (Sec. 2 Step 4 and the remark after
it) through the C ABI: the continuous reconstruction pam_eval_blend and the
interface jump pam_interface_jump, against the FP64 oracle on the same
dictionaries (built by the oracle's lattice, bit-identical to the
library's by test) and seeded coefficients.

Tolerances: FP64 queries 1e-12 relative to max|K| (rounding order of the
sums and the exp implementation); FP32 queries 2e-4 * max(1, |K|) as for
the owner reconstruction; the jump in FP64, 1e-12 relative to the largest
jump plus 1e-13. Where the answer is exact by construction it is checked
bit-for-bit against the library's own owner reconstruction: blend 0, and
points outside every band.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2605_16564_amd import api, synth  # noqa: E402
from paper_2605_16564_amd.synth import Grid  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = api.Context(0)
    yield c
    c.close()


def _t(x):
    return x.detach().cpu().numpy()


def _coefficients(od: O.Dictionary, seed):
    b = synth.random_coefficients(seed, od.n_sub, od.m_cap, od.m)
    return b, torch.as_tensor(b, device="cuda")


def _uneven3d():
    return Grid(3, [12, 10, 9], [0.0, -1.0, 0.5], [1.2, 1.0, 2.0], [3, 2, 3],
                [np.array([0, 3, 8, 12], np.int32), np.array([0, 6, 10], np.int32),
                 np.array([0, 2, 5, 9], np.int32)], 0.0, np.zeros(12 * 10 * 9))


def _special_points_2d(g):
    ax = O.grid_axis_coords(g)
    pts = []
    for a0 in ax[0]:
        for a1 in ax[1]:
            pts.append([a0, a1])                       # breakpoints, corners, domain corners
    for a0 in ax[0]:
        pts.append([a0, 0.37])
    return np.array(pts)


def _band_mask(x, axes, blend):
    inside = np.zeros(len(x), bool)
    for a, b in enumerate(axes):
        for i in range(1, len(b) - 1):
            h = blend * min(b[i] - b[i - 1], b[i + 1] - b[i])
            inside |= np.abs(x[:, a] - b[i]) < h
    return inside


@pytest.mark.parametrize("blend", [0.1, 0.5])
def test_blend_matches_oracle_2d(ctx, blend):
    g = synth.circle64(n_sub=4)
    D = api.init_lattice(ctx, g, [8, 8], m_cap=64)
    od = O.init_dictionary(g, [8, 8], 64)
    bnp, beta = _coefficients(od, 141)
    xq = np.concatenate([_special_points_2d(g),
                         synth.uniform_queries(2, 20000, seed=177, dtype=np.float64)])
    xd = torch.as_tensor(xq, device="cuda")
    out64 = api.evaluate_blend(ctx, g, D, beta, xd, blend)
    out32 = api.evaluate_blend(ctx, g, D, beta, xd.float(), blend)
    lin = api.evaluate_blend(ctx, g, D, beta, xd, blend, space=1)
    torch.cuda.synchronize()
    ref, nout = O.evaluate_blend(O.grid_axis_coords(g), od, bnp.ravel(), xq, blend)
    assert nout == 0
    scale = np.abs(ref).max()
    e64 = np.abs(_t(out64) - ref).max()
    e32 = np.abs(_t(out32).astype(np.float64) - ref).max()
    print("blend", blend, "f64 error", e64, "f32 error", e32)
    assert e64 <= 1e-12 * scale
    assert e32 <= 2e-4 * max(1.0, scale)
    assert np.allclose(_t(lin), 10.0 ** ref, rtol=1e-12)


def test_blend_matches_oracle_3d_uneven(ctx):
    g = _uneven3d()
    D = api.init_lattice(ctx, g, [3, 3, 3], m_cap=27)
    od = O.init_dictionary(g, [3, 3, 3], 27)
    bnp, beta = _coefficients(od, 142)
    rng = np.random.default_rng(143)
    lo, hi = np.array(g.lo[:3]), np.array(g.hi[:3])
    xq = lo + rng.random((30000, 3)) * (hi - lo)
    ax = O.grid_axis_coords(g)
    corners = np.array([[a, b, c] for a in ax[0] for b in ax[1] for c in ax[2]])
    xq = np.concatenate([corners, xq])
    out = api.evaluate_blend(ctx, g, D, beta, torch.as_tensor(xq, device="cuda"), 0.3)
    torch.cuda.synchronize()
    ref, nout = O.evaluate_blend(ax, od, bnp.ravel(), xq, 0.3)
    assert nout == 0
    err = np.abs(_t(out) - ref).max()
    print("3-D blend error", err)
    assert err <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_blend_reduces_to_owner_bit_for_bit(ctx, dtype):
    g = synth.circle64(n_sub=4)
    D = api.init_lattice(ctx, g, [8, 8], m_cap=64)
    od = O.init_dictionary(g, [8, 8], 64)
    _, beta = _coefficients(od, 144)
    xq = np.concatenate([_special_points_2d(g),
                         synth.uniform_queries(2, 30000, seed=145, dtype=np.float64)])
    xd = torch.as_tensor(xq, device="cuda", dtype=dtype)
    own = _t(api.evaluate(ctx, g, D, beta, xd))
    b0 = _t(api.evaluate_blend(ctx, g, D, beta, xd, 0.0))
    b2 = _t(api.evaluate_blend(ctx, g, D, beta, xd, 0.2))
    own_lin = _t(api.evaluate(ctx, g, D, beta, xd, space=1))
    b2_lin = _t(api.evaluate_blend(ctx, g, D, beta, xd, 0.2, space=1))
    assert np.array_equal(b0, own)
    keep = ~_band_mask(_t(xd).astype(np.float64), O.grid_axis_coords(g), 0.2)
    assert keep.sum() > 10000 and (~keep).sum() > 5000
    assert np.array_equal(b2[keep], own[keep])
    assert np.array_equal(b2_lin[keep], own_lin[keep])


def test_blend_multifield_and_outside(ctx):
    grids = [synth.disc_field(5100 + f, n=32 * (2 + f)) for f in range(3)]
    Ds = [api.init_lattice(ctx, g, [8, 8], m_cap=64) for g in grids]
    ods = [O.init_dictionary(g, [8, 8], 64) for g in grids]
    bs = [_coefficients(od, 160 + f) for f, od in enumerate(ods)]
    Dall = api.concat_dicts(Ds)
    ball = torch.cat([b[1] for b in bs])
    counts = [3000, 1, 2500]
    xs = [synth.uniform_queries(2, n, seed=190 + f, dtype=np.float64) for f, n in enumerate(counts)]
    xs[2][:2] = [[-0.1, 0.5], [0.5, 1.5]]            # outside the domain
    xq = torch.as_tensor(np.concatenate(xs), device="cuda")
    nout = torch.zeros(1, dtype=torch.int64, device="cuda")
    out = api.evaluate_blend(ctx, grids, Dall, ball, xq, 0.1, q_counts=counts, n_outside=nout)
    torch.cuda.synchronize()
    o = _t(out)
    assert int(nout.item()) == 2
    q0 = 0
    for f, g in enumerate(grids):
        ref, _ = O.evaluate_blend(O.grid_axis_coords(g), ods[f], bs[f][0].ravel(), xs[f], 0.1)
        got = o[q0:q0 + counts[f]]
        assert np.array_equal(np.isnan(got), np.isnan(ref))
        ok = ~np.isnan(ref)
        assert np.max(np.abs(got[ok] - ref[ok]), initial=0.0) <= 1e-12 * max(1.0, np.abs(ref[ok]).max())
        q0 += counts[f]


def test_blend_argument_errors(ctx):
    g = synth.circle64()
    D = api.init_lattice(ctx, g, [4, 4], m_cap=16)
    beta = torch.zeros(D.n_sub * 16, dtype=torch.float64, device="cuda")
    xd = torch.zeros((4, 2), dtype=torch.float64, device="cuda")
    for bad in (-0.01, 0.51, float("nan")):
        with pytest.raises(api.N.PamError):
            api.evaluate_blend(ctx, g, D, beta, xd, bad)
    with pytest.raises(api.N.PamError):
        api.interface_jump(ctx, g, D, beta, 0)
    empty = api.evaluate_blend(ctx, g, D, beta, xd[:0], 0.1)
    assert empty.numel() == 0


@pytest.mark.parametrize("case", ["2d", "3d", "multifield"])
def test_interface_jump_matches_oracle(ctx, case):
    if case == "2d":
        grids, lat, cap, n = [synth.circle64(n_sub=4)], [8, 8], 64, 16
    elif case == "3d":
        grids, lat, cap, n = [_uneven3d()], [3, 3, 3], 27, 5
    else:
        grids, lat, cap, n = [synth.disc_field(5200 + f, n=64) for f in range(2)], [8, 8], 64, 7
    Ds = [api.init_lattice(ctx, g, lat, m_cap=cap) for g in grids]
    ods = [O.init_dictionary(g, lat, cap) for g in grids]
    bs = [_coefficients(od, 170 + f) for f, od in enumerate(ods)]
    D = api.concat_dicts(Ds)
    J = _t(api.interface_jump(ctx, grids, D, torch.cat([b[1] for b in bs]), n))
    torch.cuda.synchronize()
    ref = np.concatenate([O.interface_jump(O.grid_axis_coords(g), ods[f], bs[f][0].ravel(), n)
                          for f, g in enumerate(grids)])
    assert J.shape == ref.shape == (api.interface_count(grids), 2)
    err = np.abs(J - ref).max()
    print(case, "faces", len(J), "max jump", ref[:, 0].max(), "error", err)
    assert err <= 1e-12 * ref[:, 0].max() + 1e-13
