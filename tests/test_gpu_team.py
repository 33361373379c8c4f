"""Teams of workgroups in the solve (a6): with a team, the first workgroup of
a subdomain runs the active-set iteration and the others take row slices of
its passes over the active-block inverse and the Gram. The minimizer is the
same; only summation order differs. Checked here:

  - team = 4 with sharing forced from 16 active coordinates gives the same
    coefficients as one workgroup (FP64: 1e-9, FP32 + FP64 pass: 1e-9 of
    max|beta|; both are the KKT-certified FP64 minimizer), and both match
    the FP64 oracle on sampled subdomains (the parity bars of the FP64 and
    FP32 modes);
  - a three-round refinement makes the same enrichment decisions with and
    without teams;
  - the team size reported per subdomain follows the grid that fits on the
    device (4, 2, 1), unbatched launches use one, bad values are errors;
  - members that leave early (a 1 us idle bound set from the host) have
    their rows done by the leader: the same coefficients, status OK.
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


def _grid():
    # 128 x 128 three-facies field, 4 x 4 subdomains of 32 x 32 cells
    return synth.facies256(seed=2300, n=128, n_sub=4)


def _fit(ctx, g, prec, team, team_min=16, m_cap=256):
    S = api.partition(ctx, g)
    D = api.init_lattice(ctx, g, [16, 16], m_cap)
    beta, st = api.fit(ctx, S, D, api.EnetOpts(L1, L2, prec, team=team, team_min=team_min))
    torch.cuda.synchronize()
    return _t(beta), api.stats_to_numpy(st), D


def _rel(a, b, m):
    worst = 0.0
    for s in range(len(m)):
        k = int(m[s])
        worst = max(worst, np.abs(a[s, :k] - b[s, :k]).max() / max(np.abs(b[s, :k]).max(), 1e-300))
    return worst


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_team_matches_one_workgroup_and_oracle(ctx, prec):
    g = _grid()
    b1, st1, D = _fit(ctx, g, prec, team=1)
    b4, st4, _ = _fit(ctx, g, prec, team=4)
    m = _t(D.m)
    print(prec, "support max", st4["support"].max(), "teams", np.unique(st4["team"]),
          "kkt", st1["kkt"].max(), st4["kkt"].max())
    assert np.all(st1["status"] == 0) and np.all(st4["status"] == 0)
    assert np.all(st1["team"] == 1) and np.all(st4["team"] == 4)
    assert st4["support"].max() >= 64          # the shared passes did run
    assert st4["kkt"].max() <= 1e-9 and st1["kkt"].max() <= 1e-9
    err = _rel(b4, b1, m)
    print("team vs one workgroup", err)
    assert err <= 1e-9
    # sampled subdomains against the FP64 oracle
    od = O.init_dictionary(g, [16, 16], 256)
    op = O.partition(g)
    for s in (0, 9):
        lo, hi = int(op["off"][s]), int(op["off"][s + 1])
        k = int(od.m[s])
        c = od.c[s * 256 * 2:(s * 256 + k) * 2].reshape(k, 2)
        sg = od.sigma[s * 256:s * 256 + k]
        bo, sto, _ = O.fit_one(op["x"][lo:hi], op["y"][lo:hi], c, sg, L1, L2)
        e = np.abs(b4[s, :k] - bo).max() / np.abs(bo).max()
        print("subdomain", s, "oracle error", e)
        assert sto == 0 and e <= (1e-9 if prec == "f64" else 1e-5)


def test_team_refinement_decisions(ctx):
    g = _grid()
    out = []
    for team in (1, 4):
        S = api.partition(ctx, g)
        D = api.init_lattice(ctx, g, [12, 12], 720)
        eps = 1e-4 * float(np.prod(g.cell_size))
        beta, lvl, rounds, rs, st = api.refine(
            ctx, S, D, api.EnetOpts(L1, L2, "f32", team=team, team_min=16),
            api.RefineOpts(k_top=64, max_rounds=3, eps_tol=eps))
        torch.cuda.synchronize()
        stn = api.stats_to_numpy(st)
        assert np.all(stn["status"] == 0) and stn["kkt"].max() <= 1e-9
        out.append((_t(beta), _t(D.m), _t(D.c), _t(lvl), _t(rounds)))
    (b1, m1, c1, l1, r1), (b4, m4, c4, l4, r4) = out
    print("centers", m1.sum(), m4.sum(), "rounds", r1.sum(), r4.sum())
    assert np.array_equal(m1, m4) and np.array_equal(r1, r4) and np.array_equal(l1, l4)
    assert np.array_equal(c1, c4)
    assert _rel(b4, b1, m1) <= 1e-9


def test_team_size_follows_the_resident_grid(ctx):
    g = _grid()                                   # 16 subdomains
    _, st, _ = _fit(ctx, g, "f64", team=0, team_min=0)
    assert np.all(st["team"] == 4)
    _, st, _ = _fit(ctx, g, "f64", team=2, team_min=0)
    assert np.all(st["team"] == 2)
    g100 = synth.facies256(seed=2301, n=320, n_sub=10)   # 100 subdomains: 400 > 256 CUs
    S = api.partition(ctx, g100)
    D = api.init_lattice(ctx, g100, [8, 8], 64)
    beta, st = api.fit(ctx, S, D, api.EnetOpts(L1, L2, "f64"))
    stn = api.stats_to_numpy(st)
    print("100 subdomains: team", np.unique(stn["team"]))
    assert np.all(stn["status"] == 0) and np.all(stn["team"] == 2)
    S = api.partition(ctx, g)
    D = api.init_lattice(ctx, g, [8, 8], 64)
    beta, st = api.fit(ctx, S, D, api.EnetOpts(L1, L2, "f64", batched=False))
    assert np.all(api.stats_to_numpy(st)["team"] == 1)
    for bad in (dict(team=3), dict(team=-1), dict(team_min=-2), dict(team_idle_us=-1),
                dict(team_idle_us=10_000_001)):
        with pytest.raises(api.N.PamError):
            api.fit(ctx, S, D, api.EnetOpts(L1, L2, "f64", **bad))


def test_members_that_leave_are_replaced_by_the_leader(ctx):
    g = _grid()
    S = api.partition(ctx, g)
    D = api.init_lattice(ctx, g, [16, 16], 256)
    ref, st1 = api.fit(ctx, S, D, api.EnetOpts(L1, L2, "f64", team=1))
    out, st4 = api.fit(ctx, S, D, api.EnetOpts(L1, L2, "f64", team=4, team_min=16, team_idle_us=1))
    torch.cuda.synchronize()
    s1, s4 = api.stats_to_numpy(st1), api.stats_to_numpy(st4)
    assert np.all(s4["status"] == 0) and np.all(s4["team"] == 4)
    assert s4["kkt"].max() <= 1e-9
    err = _rel(_t(out), _t(ref), _t(D.m))
    print("members left early: coefficients vs one workgroup", err)
    assert err <= 1e-9
