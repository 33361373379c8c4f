"""GPU parity of the Darcy consumer (pam_darcy_solve, pam_darcy_error; Sec. 5
Eq. (darcy_model), Exp. 1's pressure experiment, Eq. (pressure_L2_error))
against the FP64 oracle (element-by-element P1 assembly, sparse direct
solve, exact P1 mass matrix), through the C ABI.

Tolerances: the GPU solve stops at ||r|| <= 1e-12 ||b||; nodal pressures
within 1e-8 (absolute, pressures in [0, 1]) of the direct solve for
contrasts up to 1e6; the relative error norm 1e-12 relative; closed-form
cases (constant K, layers along the flow) exact to 1e-10.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import darcy_oracle as DO  # noqa: E402
from oracle import oracle as O  # noqa: E402
from paper_2605_16564_amd import api, synth  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = api.Context(0)
    yield c
    c.close()


def _t(x):
    return x.detach().cpu().numpy()


def _opts(n0, n1, lo=(0.0, 0.0), hi=(1.0, 1.0), **kw):
    return api.DarcyOpts(n0, n1, lo, hi, tol=kw.pop("tol", 1e-12), **kw)


def test_solve_matches_direct_solve(ctx):
    o = _opts(48, 40, (0.5, -1.0), (2.0, 1.0))
    rng = np.random.default_rng(11)
    k = 10.0 ** rng.uniform(-3, 3, size=(40, 48, 2))
    p, it, res = api.darcy_solve(ctx, o, torch.as_tensor(k, device="cuda"))
    ref = DO.solve(48, 40, np.array(o.lo), np.array(o.hi), k)
    err = np.abs(_t(p) - ref).max()
    print("iterations", it, "residual", res, "max error", err)
    assert res <= 1e-12 and err <= 1e-8


def test_closed_forms(ctx):
    o = _opts(20, 12, (0.0, 0.0), (3.0, 1.0), p_left=2.0, p_right=-1.0)
    X = DO.nodes(20, 12, np.array(o.lo), np.array(o.hi))
    lin = 2.0 - 3.0 * X[:, 0] / 3.0
    rng = np.random.default_rng(12)
    layers = 10.0 ** rng.uniform(-2, 2, size=12)
    for k in (np.full((12, 20, 2), 0.3), np.broadcast_to(layers[:, None, None], (12, 20, 2)).copy()):
        p, it, res = api.darcy_solve(ctx, o, torch.as_tensor(k, device="cuda"))
        assert np.abs(_t(p) - lin).max() <= 1e-10


def test_error_norm_matches_oracle(ctx):
    o = _opts(30, 22, (0.0, 1.0), (1.5, 2.0))
    rng = np.random.default_rng(13)
    a, b = rng.random(31 * 23), rng.random(31 * 23)
    e = api.darcy_error(ctx, o, torch.as_tensor(a, device="cuda"), torch.as_tensor(b, device="cuda"))
    ref = DO.relative_error(30, 22, np.array(o.lo), np.array(o.hi), a, b)
    assert abs(e - ref) <= 1e-12 * ref
    assert api.darcy_error(ctx, o, torch.as_tensor(a, device="cuda"),
                           torch.as_tensor(a, device="cuda")) == 0.0


def test_warm_start_and_errors(ctx):
    o = _opts(24, 24)
    rng = np.random.default_rng(14)
    k = torch.as_tensor(10.0 ** rng.uniform(-1, 1, size=(24, 24, 2)), device="cuda")
    p, it, res = api.darcy_solve(ctx, o, k)
    p2, it2, res2 = api.darcy_solve(ctx, o, k, p=p.clone())
    assert it > o.check_every and it2 <= o.check_every and res2 <= 1e-12
    for bad in (dict(n0=0), dict(tol=0.0), dict(check_every=0), dict(hi=(0.0, 1.0))):
        kw = dict(n0=24, n1=24, lo=(0.0, 0.0), hi=(1.0, 1.0), tol=1e-12)
        kw.update(bad)
        with pytest.raises(api.N.PamError):
            api.darcy_solve(ctx, api.DarcyOpts(**kw), k)


def test_reconstruction_to_pressure_error(ctx):
    """Fitted circle field -> K* at the triangle centroids -> pressure, against
    the oracle's own chain (its fit, its evaluation, its assembly and solve);
    E_p against the pressure of the data's own coefficient."""
    g = synth.circle64()
    S = api.partition(ctx, g)
    D = api.init_lattice(ctx, g, [16, 16], m_cap=256)
    beta, _ = api.fit(ctx, S, D, api.EnetOpts(synth.LAMBDA1, synth.LAMBDA2, "f64"))
    o = _opts(64, 64)
    k_star = api.darcy_k_from_reconstruction(ctx, g, D, beta, o)
    k_true = api.darcy_k_from_cells(ctx, g, o)
    p_star, it1, _ = api.darcy_solve(ctx, o, k_star)
    p_true, it2, _ = api.darcy_solve(ctx, o, k_true)
    e_gpu = api.darcy_error(ctx, o, p_true, p_star)
    od = O.init_dictionary(g, [16, 16], 256)
    bo, _, _ = O.fit_batch(O.partition(g), od, synth.LAMBDA1, synth.LAMBDA2)
    lo, hi = np.zeros(2), np.ones(2)
    cen = DO.centroids(64, 64, lo, hi).reshape(-1, 2)
    ks_o = O.evaluate(O.grid_axis_coords(g), od, bo, cen, space=1)[0].reshape(64, 64, 2)
    kt_o = DO.k_from_cells(64, 64, lo, hi, g.y, 64, 64)
    assert np.abs(_t(k_true) - kt_o).max() <= 1e-15 * kt_o.max()
    assert np.abs(_t(k_star) - ks_o).max() <= 1e-8 * ks_o.max()
    ps_o = DO.solve(64, 64, lo, hi, ks_o)
    pt_o = DO.solve(64, 64, lo, hi, kt_o)
    e_o = DO.relative_error(64, 64, lo, hi, pt_o, ps_o)
    print("E_p gpu", e_gpu, "oracle", e_o, "iterations", it1, it2)
    assert np.abs(_t(p_star) - ps_o).max() <= 1e-8
    assert np.abs(_t(p_true) - pt_o).max() <= 1e-8
    assert abs(e_gpu - e_o) <= 1e-6 * e_o


def test_graph_bursts_replay_the_eager_iteration(ctx):
    """Full bursts run as replays of one executable graph, a shorter last
    burst as separate launches; the same 256 iterations both ways (4 graph
    replays with host synchronizations between them, against 256 eager
    iterations) give bit-identical pressures."""
    rng = np.random.default_rng(15)
    k = torch.as_tensor(10.0 ** rng.uniform(-2, 2, size=(40, 40, 2)), device="cuda")
    g = api.DarcyOpts(40, 40, tol=1e-300, max_iter=256, check_every=64)
    e = api.DarcyOpts(40, 40, tol=1e-300, max_iter=256, check_every=1000)
    pg, itg, _ = api.darcy_solve(ctx, g, k)
    pe, ite, _ = api.darcy_solve(ctx, e, k)
    pg2, _, _ = api.darcy_solve(ctx, g, k)
    assert itg == ite == 256
    assert torch.equal(pg, pe) and torch.equal(pg, pg2)
