"""GPU parity of the per-subdomain elastic-net parameter choice
(pam_select_lambda: alpha path + K-fold cross-validation; Sec. 2 after Eq.
(elastic), Exp. 1.2) against the FP64 oracle, through the C ABI.

Tolerances: the path's alpha_max in FP64 on both sides, 1e-12 relative;
scores are held-out errors of FP64 minimizers (every precision mode ends on
the FP64 problem), 1e-7 relative to the largest score plus 1e-12; the
chosen index must equal the oracle's unless the oracle's own scores at the
two choices are within that tolerance (then both are correct). Refits with
the chosen per-subdomain parameters: coefficients 1e-9 of max|beta| (FP64).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

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


def _compare(out, ref, tol=1e-7):
    alpha, score, best, l1, l2 = ref
    ga, gs, gb = _t(out["alpha"]), _t(out["score"]), _t(out["best"])
    assert np.abs(ga - alpha).max() <= 1e-12 * max(np.abs(alpha).max(), 1e-300)
    serr = np.abs(gs - score).max()
    stol = tol * np.abs(score).max() + 1e-12
    assert serr <= stol, serr
    for s in range(len(best)):
        if gb[s] != best[s]:
            assert abs(score[s, gb[s]] - score[s, best[s]]) <= stol, (s, gb[s], best[s])
    a_g = ga[np.arange(len(gb)), gb]
    assert np.array_equal(_t(out["lambda1"]), 0.99 * a_g)
    assert np.array_equal(_t(out["lambda2"]), (1 - 0.99) * a_g)
    assert np.all(_t(out["n_failed"]) == 0)
    return serr, int((gb != best).sum())


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_select_matches_oracle_circle(ctx, prec):
    g = synth.circle64()
    S = api.partition(ctx, g)
    D = api.init_lattice(ctx, g, [6, 6], m_cap=36)
    opts = api.EnetOpts(0.0, 0.0, prec)
    out = api.select_lambda(ctx, S, D, opts, n_alpha=6, k_folds=4, alpha_min_ratio=1e-3)
    torch.cuda.synchronize()
    ref = O.select_lambda(O.partition(g), O.init_dictionary(g, [6, 6], 36), n_alpha=6, ratio=1e-3,
                          k_folds=4)
    serr, moved = _compare(out, ref)
    print(prec, "score error", serr, "best", _t(out["best"]), "oracle", ref[2], "moved", moved)


def test_select_matches_oracle_facies_and_refit(ctx):
    g = synth.facies256(n=64, n_sub=4)
    S = api.partition(ctx, g)
    D = api.init_lattice(ctx, g, [8, 8], m_cap=64)
    out = api.select_lambda(ctx, S, D, api.EnetOpts(0.0, 0.0, "f64"), n_alpha=8, k_folds=5)
    torch.cuda.synchronize()
    Sn = O.partition(g)
    od = O.init_dictionary(g, [8, 8], 64)
    ref = O.select_lambda(Sn, od, n_alpha=8, ratio=1e-3, k_folds=5)
    serr, moved = _compare(out, ref)
    print("facies score error", serr, "moved", moved, "chosen", np.bincount(ref[2], minlength=8))
    # refit on all samples with the chosen per-subdomain parameters
    opts = api.EnetOpts(0.0, 0.0, "f64", lambda1_sub=out["lambda1"], lambda2_sub=out["lambda2"])
    beta, st = api.fit(ctx, S, D, opts)
    torch.cuda.synchronize()
    l1g, l2g = _t(out["lambda1"]), _t(out["lambda2"])
    worst = 0.0
    for s in range(od.n_sub):
        j0, j1 = Sn["off"][s], Sn["off"][s + 1]
        c = od.c[s * 64 * 2:(s + 1) * 64 * 2].reshape(64, 2)
        sg = od.sigma[s * 64:(s + 1) * 64]
        bo, status, _ = O.fit_one(Sn["x"][j0:j1], Sn["y"][j0:j1], c, sg, l1g[s], l2g[s])
        assert status == 0
        err = np.abs(_t(beta)[s] - bo).max() / max(np.abs(bo).max(), 1e-300)
        worst = max(worst, err)
    print("refit coefficient error", worst)
    assert worst <= 1e-9
    assert np.all(api.stats_to_numpy(st)["status"] == 0)


def test_select_with_more_centers_than_training_samples(ctx):
    g = synth.facies256(n=32, n_sub=4)           # 8 x 8 cells per subdomain
    S = api.partition(ctx, g)
    D = api.init_lattice(ctx, g, [12, 12], m_cap=144)
    out = api.select_lambda(ctx, S, D, api.EnetOpts(0.0, 0.0, "f64"), n_alpha=5, k_folds=4,
                            alpha_min_ratio=1e-2)
    torch.cuda.synchronize()
    ref = O.select_lambda(O.partition(g), O.init_dictionary(g, [12, 12], 144), n_alpha=5,
                          ratio=1e-2, k_folds=4)
    serr, moved = _compare(out, ref)
    print("M > N score error", serr, "moved", moved)


def test_select_argument_errors(ctx):
    g = synth.circle64(n=32, n_sub=2)
    S = api.partition(ctx, g)
    D = api.init_lattice(ctx, g, [3, 3], m_cap=9)
    o = api.EnetOpts(0.0, 0.0, "f64")
    for kw in (dict(n_alpha=0), dict(k_folds=1), dict(alpha_min_ratio=0.0),
               dict(alpha_min_ratio=1.5), dict(l1_ratio=0.0)):
        with pytest.raises(api.N.PamError):
            api.select_lambda(ctx, S, D, o, **kw)
    out = api.select_lambda(ctx, S, D, o, n_alpha=1, k_folds=2)
    torch.cuda.synchronize()
    assert np.all(_t(out["best"]) == 0)
