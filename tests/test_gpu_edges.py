"""Edge cases of the fit through the C ABI: more centers than samples (the
elastic net stays strictly convex through lambda2), subdomains without
centers, the largest dictionary the LDS-resident solve accepts and the
capacity error just past it."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2605_16564_amd import api, native, synth  # noqa: E402

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


def _dict_from(od):
    D = api.Dictionary.empty(od.n_sub, od.dim, od.m_cap, torch.device("cuda"))
    D.m.copy_(torch.as_tensor(od.m))
    D.c.copy_(torch.as_tensor(od.c.reshape(od.n_sub, od.m_cap, od.dim)))
    D.sigma.copy_(torch.as_tensor(od.sigma.reshape(od.n_sub, od.m_cap)))
    D.level.copy_(torch.as_tensor(od.level.reshape(od.n_sub, od.m_cap)))
    return D


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_more_centers_than_samples(ctx, prec):
    """2x2 subdomains of 16x16 cells (N = 256) with a 24x24 lattice (M = 576):
    underdetermined least squares, unique elastic-net minimizer."""
    g = synth.facies256(seed=2005, n=32, n_sub=2)
    S = api.partition(ctx, g)
    D = api.init_lattice(ctx, g, [24, 24], 600)
    beta, st = api.fit(ctx, S, D, api.EnetOpts(L1, L2, prec))
    torch.cuda.synchronize()
    stn = api.stats_to_numpy(st)
    assert np.all(stn["status"] == 0) and stn["kkt"].max() < 1e-9, stn["kkt"]
    od = O.init_dictionary(g, [24, 24], 600)
    bo, sto, _ = O.fit_batch(O.partition(g), od, L1, L2)
    b = _t(beta)
    err = max(np.abs(b[s, :576] - bo[s * 600:s * 600 + 576]).max() / np.abs(bo[s * 600:s * 600 + 576]).max()
              for s in range(4))
    print(prec, "M > N coefficient error", err, "support", stn["support"])
    assert err <= (1e-9 if prec == "f64" else 1e-5)


def test_subdomains_without_centers(ctx):
    g = synth.circle64()
    S = api.partition(ctx, g)
    od = O.init_dictionary(g, [16, 16], 256)
    od.m[1] = 0
    od.m[3] = 0
    D = _dict_from(od)
    beta = torch.full((4, 256), 7.0, dtype=torch.float64, device="cuda")   # cold fit overwrites
    beta, st = api.fit(ctx, S, D, api.EnetOpts(L1, L2, "f64"))
    torch.cuda.synchronize()
    stn = api.stats_to_numpy(st)
    assert list(stn["status"]) == [0, native.ST_EMPTY, 0, native.ST_EMPTY]
    b = _t(beta)
    assert np.all(b[1] == 0.0) and np.all(b[3] == 0.0)
    bo, _, _ = O.fit_batch(O.partition(g), O.init_dictionary(g, [16, 16], 256), L1, L2)
    for s in (0, 2):
        ref = bo[s * 256:(s + 1) * 256]
        assert np.abs(b[s] - ref).max() <= 1e-9 * np.abs(ref).max()


def test_largest_dictionary_and_capacity_error(ctx):
    """The solve keeps 57 B per center in LDS beside about 20 KB of fixed
    state, within 160 KiB per workgroup: a 48x48 lattice (2304 centers, m_cap
    2304) on one 64x64-cell subdomain fits; m_cap = 2720 is refused with a
    capacity error before anything runs."""
    g = synth.facies256(seed=2006, n=64, n_sub=1)
    S = api.partition(ctx, g)
    D = api.init_lattice(ctx, g, [48, 48], 2304)
    beta, st = api.fit(ctx, S, D, api.EnetOpts(L1, L2, "f32"))
    torch.cuda.synchronize()
    stn = api.stats_to_numpy(st)
    print("M = 2304: status", stn["status"], "kkt", stn["kkt"], "support", stn["support"])
    assert stn["status"][0] == 0 and stn["kkt"][0] < 1e-9
    Dbig = api.init_lattice(ctx, g, [48, 48], 2720)
    with pytest.raises(native.PamError, match="m_cap too large"):
        api.fit(ctx, S, Dbig, api.EnetOpts(L1, L2, "f32"))


def test_nonfinite_input_detected(ctx):
    """A NaN data value, an infinite sample point, an infinite center or a
    zero width leaves that subdomain unfitted with status NONFINITE (beta
    zero) while the others are fitted as usual; pam_sync then reports
    PAM_ERR_NONFINITE once (the flag is sticky until read)."""
    g = synth.circle64()
    S = api.partition(ctx, g)
    od = O.init_dictionary(g, [16, 16], 256)
    bo, _, _ = O.fit_batch(O.partition(g), od, L1, L2)
    ctx.sync()                                   # clears any earlier flag
    for case in ("nan_y", "inf_x", "inf_c", "zero_sigma", "inf_y_refine"):
        print("case", case, flush=True)
        S2 = api.Samples(S.dim, S.n_sub, S.n_max, S.off, S.off_host, S.x.clone(), S.y.clone(),
                         S.h.clone())
        D = _dict_from(od if case != "inf_y_refine" else O.init_dictionary(g, [16, 16], 556))
        j = int(S.off_host[1]) + 17              # an element of subdomain 1
        if case == "nan_y":
            S2.y[j] = float("nan")
        elif case == "inf_x":
            S2.x[j, 0] = float("inf")
        elif case == "inf_c":
            D.c[1, 5, 1] = float("-inf")
        elif case == "zero_sigma":
            D.sigma[1, 9] = 0.0
        else:
            S2.y[j] = float("inf")
        if case == "inf_y_refine":
            beta, lvl, rounds, rs, st = api.refine(ctx, S2, D, api.EnetOpts(L1, L2, "f64"),
                                                   api.RefineOpts(k_top=50, max_rounds=2,
                                                                  eps_tol=1e-9))
        else:
            beta = torch.full((4, 256), 7.0, dtype=torch.float64, device="cuda")
            beta, st = api.fit(ctx, S2, D, api.EnetOpts(L1, L2, "f64"))
        with pytest.raises(native.PamError) as ei:
            ctx.sync()
        assert ei.value.status == native.ERR_NONFINITE
        ctx.sync()                               # read once: cleared
        stn = api.stats_to_numpy(st)
        assert stn["status"][1] == native.ST_NONFINITE
        assert np.all(np.delete(stn["status"], 1) == 0)
        b = _t(beta)
        assert np.all(b[1] == 0.0)
        if case == "inf_y_refine":
            assert int(_t(D.m).min()) == 256 and int(_t(D.m).max()) > 256
            r = _t(rounds)
            assert r[1] == 1 and np.all(np.delete(r, 1) >= 2)
            assert int(_t(D.m)[1]) == 256        # not enriched
            continue
        for s in (0, 2, 3):
            ref = bo[s * 256:(s + 1) * 256]
            assert np.abs(b[s] - ref).max() <= 1e-9 * np.abs(ref).max()
