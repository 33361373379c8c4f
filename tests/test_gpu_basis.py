"""GPU parity of the ablations the paper describes, through the C ABI against
the FP64 oracle: the plain (unnormalized) basis of Example 1 (Sec. 3.2) --
fits in FP64 and FP32 modes, a two-round refinement and the evaluation --
and the indicator measured on K itself instead of log10 K (Alg. 1 literal).

Tolerances as for the Shepard basis: FP64 coefficients 1e-9 of max|beta|,
FP32 mode 1e-5, refinement dictionaries and levels bit-exact, FP64
evaluation 1e-12 of max|K|.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2605_16564_amd import api, synth  # noqa: E402

L1, L2 = synth.LAMBDA1, synth.LAMBDA2


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = api.Context(0)
    yield c
    c.close()


def _t(x):
    return x.detach().cpu().numpy()


def _coef_err(beta_gpu, bo, m, m_cap):
    worst = 0.0
    for s in range(len(m)):
        ref = bo[s * m_cap:s * m_cap + int(m[s])]
        worst = max(worst, np.abs(beta_gpu[s, :int(m[s])] - ref).max() / np.abs(ref).max())
    return worst


@pytest.mark.parametrize("prec,tol", [("f64", 1e-9), ("f32", 1e-5)])
def test_plain_fit_matches_oracle(ctx, prec, tol):
    g = synth.circle64()
    S = api.partition(ctx, g)
    D = api.init_lattice(ctx, g, [12, 12], m_cap=144, basis="plain")
    beta, st = api.fit(ctx, S, D, api.EnetOpts(L1, L2, prec))
    torch.cuda.synchronize()
    od = O.init_dictionary(g, [12, 12], 144, basis="plain")
    bo, sto, _ = O.fit_batch(O.partition(g), od, L1, L2)
    err = _coef_err(_t(beta), bo, od.m, 144)
    stn = api.stats_to_numpy(st)
    print(prec, "plain basis coefficient error", err, "kkt", stn["kkt"].max())
    assert np.all(stn["status"] == 0) and np.all(sto == 0)
    assert err <= tol
    # a different problem from the Shepard fit of the same data
    bs, _ = api.fit(ctx, S, api.init_lattice(ctx, g, [12, 12], m_cap=144),
                    api.EnetOpts(L1, L2, prec))
    assert _t((bs - beta).abs().max()) > 1e-3


def test_plain_refine_and_eval_match_oracle(ctx):
    g = synth.facies256(n=64, n_sub=4)
    S = api.partition(ctx, g)
    m_cap = 64 + 2 * 3 * 51
    D = api.init_lattice(ctx, g, [8, 8], m_cap=m_cap, basis="plain")
    tol = 1e-4 * (1 / 64) ** 2
    beta, lvl, rounds, rs, st = api.refine(ctx, S, D, api.EnetOpts(L1, L2, "f64"),
                                           api.RefineOpts(k_top=51, max_rounds=2, eps_tol=tol))
    xq = synth.uniform_queries(2, 20000, seed=620, dtype=np.float64)
    out = api.evaluate(ctx, g, D, beta, torch.as_tensor(xq, device="cuda"))
    torch.cuda.synchronize()
    od = O.init_dictionary(g, [8, 8], m_cap, basis="plain")
    odr, bo, lvo, info = O.refine_batch(O.partition(g), od, L1, L2, k_top=51, max_rounds=2,
                                        m_max=1 << 30, eps_tol=tol)
    assert np.array_equal(_t(D.m), odr.m)
    assert np.array_equal(_t(lvl), lvo)
    err = _coef_err(_t(beta), bo, odr.m, m_cap)
    ref, _ = O.evaluate(O.grid_axis_coords(g), odr, bo, xq)
    eerr = np.abs(_t(out) - ref).max()
    print("plain refine coefficient error", err, "eval error", eerr, "centers", _t(D.m))
    assert err <= 1e-9
    assert eerr <= 1e-8 * np.abs(ref).max()


def test_unknown_basis_is_rejected(ctx):
    g = synth.circle64(n=32, n_sub=2)
    S = api.partition(ctx, g)
    D = api.init_lattice(ctx, g, [3, 3], m_cap=9)
    D.basis = "other"
    with pytest.raises(api.N.PamError):
        api.fit(ctx, S, D, api.EnetOpts(L1, L2, "f64"))


def test_linear_space_indicator_refine_matches_oracle(ctx):
    g = synth.facies256(n=64, n_sub=4)
    S = api.partition(ctx, g)
    m_cap = 64 + 2 * 3 * 51
    D = api.init_lattice(ctx, g, [8, 8], m_cap=m_cap)
    tol = 1e-3 * (1 / 64) ** 2
    beta, lvl, rounds, rs, st = api.refine(ctx, S, D, api.EnetOpts(L1, L2, "f64"),
                                           api.RefineOpts(k_top=51, max_rounds=2, eps_tol=tol,
                                                          space=1))
    torch.cuda.synchronize()
    od = O.init_dictionary(g, [8, 8], m_cap)
    odr, bo, lvo, info = O.refine_batch(O.partition(g), od, L1, L2, k_top=51, max_rounds=2,
                                        m_max=1 << 30, eps_tol=tol, space=1)
    assert np.array_equal(_t(D.m), odr.m)
    assert np.array_equal(_t(lvl), lvo)
    assert np.array_equal(_t(rounds), info["rounds"])
    err = _coef_err(_t(beta), bo, odr.m, m_cap)
    print("linear-space indicator refine coefficient error", err, "centers", _t(D.m))
    assert err <= 1e-9
