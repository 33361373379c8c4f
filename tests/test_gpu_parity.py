"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances (FP64 path): coefficients 1e-9 relative to max|beta| (both sides
solve the same strictly convex problem; they differ only in rounding order
and exp implementation, amplified by the conditioning of the active block),
supports equal on every coordinate whose oracle KKT margin exceeds
1e-9 * max(lambda1, max|beta|); integer work (samples, dictionaries, levels)
bit-exact.
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


def _coefficients(od: O.Dictionary, seed):
    """Seeded coefficients for the evaluation tests (same values on both sides)."""
    b = synth.random_coefficients(seed, od.n_sub, od.m_cap, od.m)
    return b, torch.as_tensor(b, device="cuda")


def _margins(x, y, c, sig, beta, l1, l2):
    W = O.design(x, c, sig)
    G, b = O.normal(W, y)
    g = b - G @ beta - l2 * beta
    return np.where(beta != 0, np.abs(beta), l1 - np.abs(g)), G, b


def _check_fit(S, D, beta_gpu, beta_ora, l1, l2, rel_tol):
    off = S["off"]
    m = D.m
    worst = 0.0
    for s in range(D.n_sub):
        M = int(m[s])
        bg = beta_gpu[s, :M]
        bo = beta_ora[s * D.m_cap: s * D.m_cap + M]
        scale = max(np.abs(bo).max(), 1e-300)
        err = np.abs(bg - bo).max() / scale
        worst = max(worst, err)
        assert err <= rel_tol, (s, err)
        assert np.all(beta_gpu[s, M:] == 0.0)
        x = S["x"][off[s]:off[s + 1]]
        y = S["y"][off[s]:off[s + 1]]
        c = D.c[s * D.m_cap * D.dim:(s * D.m_cap + M) * D.dim].reshape(M, D.dim)
        sg = D.sigma[s * D.m_cap:s * D.m_cap + M]
        marg, G, b = _margins(x, y, c, sg, bo, l1, l2)
        firm = marg > 1e-9 * max(l1, scale)
        assert np.array_equal((bg != 0)[firm], (bo != 0)[firm]), s
    return worst


# ---------------------------------------------------------------- a1, a2
@pytest.mark.parametrize("make", [lambda: synth.circle64(),
                                  lambda: synth.layered3d(nx=12, ny=10, nz=17, sub=(2, 2, 3)),
                                  lambda: synth.disc_field(5003), lambda: synth.step1d(64)])
def test_partition_and_lattice_bit_exact(ctx, make):
    g = make()
    print("case", g.dim, g.n_cells, g.n_sub, flush=True)
    S = api.partition(ctx, g)
    ref = O.partition(g)
    torch.cuda.synchronize()
    assert np.array_equal(S.off_host, ref["off"])
    assert np.array_equal(_t(S.x), ref["x"])
    assert np.array_equal(_t(S.y), ref["y"])
    assert np.array_equal(_t(S.h), ref["h"])
    assert np.array_equal(_t(S.cell), ref["cell"])
    glat = [4, 3, 2][: g.dim]
    D = api.init_lattice(ctx, g, glat, m_cap=40)
    od = O.init_dictionary(g, glat, 40)
    torch.cuda.synchronize()
    M = int(np.prod(glat))
    assert np.all(_t(D.m) == M)
    gc = _t(D.c)[:, :M]
    oc = od.c.reshape(D.n_sub, 40, g.dim)[:, :M]
    bad = np.argwhere(gc != oc)
    if len(bad):
        s_, k_, a_ = bad[0]
        print("first lattice mismatch", bad[0], repr(gc[s_, k_, a_]), repr(oc[s_, k_, a_]),
              "count", len(bad), flush=True)
    assert len(bad) == 0
    assert np.array_equal(_t(D.sigma)[:, :M], od.sigma.reshape(D.n_sub, 40)[:, :M])
    assert np.all(_t(D.level)[:, :M] == 0)


# ---------------------------------------------------------------- a3-a6
def _ragged_grid():
    rng = np.random.default_rng(9)
    y = np.where(rng.random((40, 48)) < 0.5, -1.0, 2.0)
    y[:, 20:] += 1.0
    return synth.Grid(2, [48, 40, 1], [0.0, 0.0, 0.0], [1.2, 1.0, 1.0], [3, 2, 1],
                      [np.array([0, 13, 30, 48], np.int32), np.array([0, 17, 40], np.int32),
                       np.array([0, 1], np.int32)], 0.1, y.ravel())


@pytest.mark.parametrize("case", ["circle64", "ragged", "step1d"])
def test_fit_f64_matches_oracle(ctx, case):
    if case == "circle64":
        g, lat, cap = synth.circle64(), [16, 16], 256
    elif case == "ragged":
        g, lat, cap = _ragged_grid(), [7, 6], 50
    else:
        g, lat, cap = synth.step1d(64), [9], 9
    print("case", case, flush=True)
    S = api.partition(ctx, g)
    D = api.init_lattice(ctx, g, lat, m_cap=cap)
    opts = api.EnetOpts(L1, L2, "f64", cd_sweeps=8)
    beta, stats = api.fit(ctx, S, D, opts)
    torch.cuda.synchronize()
    st = api.stats_to_numpy(stats)
    assert np.all(st["status"] == 0), st
    assert np.all(st["kkt"] < 1e-10), st["kkt"]
    Sn = O.partition(g)
    od = O.init_dictionary(g, lat, cap)
    bo, sto, _ = O.fit_batch(Sn, od, L1, L2, cd_sweeps=8)
    assert np.all(sto == 0)
    worst = _check_fit(Sn, od, _t(beta), bo, L1, L2, 1e-9)
    print("max rel coefficient error", worst)


def test_fit_warm_start_hint_and_unbatched_agree(ctx):
    g = _ragged_grid()
    S = api.partition(ctx, g)
    D = api.init_lattice(ctx, g, [7, 6], m_cap=50)
    b1, _ = api.fit(ctx, S, D, api.EnetOpts(L1, L2, "f64", cd_sweeps=8))
    b2, _ = api.fit(ctx, S, D, api.EnetOpts(L1, L2, "f64", cd_sweeps=8))
    b3, _ = api.fit(ctx, S, D, api.EnetOpts(L1, L2, "f64", cd_sweeps=8, batched=False))
    b4, st4 = api.fit(ctx, S, D, api.EnetOpts(L1, L2, "f64", cd_sweeps=0),
                      beta=torch.randn_like(b1) * (torch.arange(50, device=b1.device) < 42))
    hint = (b1 != 0).to(torch.uint8)
    b5, st5 = api.fit(ctx, S, D, api.EnetOpts(L1, L2, "f64", cd_sweeps=0, support_hint=hint))
    torch.cuda.synchronize()
    assert torch.equal(b1, b2)                      # deterministic
    assert torch.equal(b1, b3)                      # batching does not change results
    for b in (b4, b5):
        err = (b - b1).abs().max().item() / b1.abs().max().item()
        assert err < 1e-9
    # starting from the exact support needs no more iterations than a cold start
    cold = api.stats_to_numpy(api.fit(ctx, S, D, api.EnetOpts(L1, L2, "f64", cd_sweeps=0))[1])
    assert np.all(api.stats_to_numpy(st5)["iters"] <= cold["iters"])


def test_fit_edge_cases(ctx):
    g = _ragged_grid()
    S = api.partition(ctx, g)
    D = api.init_lattice(ctx, g, [7, 6], m_cap=50)
    # lambda1 above ||b||_inf: exactly zero
    b, st = api.fit(ctx, S, D, api.EnetOpts(1e6, L2, "f64"))
    torch.cuda.synchronize()
    assert torch.count_nonzero(b).item() == 0
    assert np.all(api.stats_to_numpy(st)["status"] == 0)
    # one center per subdomain: beta = Shepard average of y (ridge on a constant column)
    D1 = api.init_lattice(ctx, g, [1, 1], m_cap=4)
    b1, _ = api.fit(ctx, S, D1, api.EnetOpts(0.0, 0.0, "f64"))
    torch.cuda.synchronize()
    yv = _t(S.y)
    for s in range(D1.n_sub):
        ys = yv[S.off_host[s]:S.off_host[s + 1]]
        assert abs(_t(b1)[s, 0] - ys.mean()) < 1e-12 * max(1, abs(ys.mean()))


# ---------------------------------------------------------------- a7-a9
def test_refine_matches_oracle_small(ctx):
    """Alg. 1 on a 64x64 facies field, 4x4 subdomains of 16x16 elements, 8x8
    initial centers, K_top = 51, three enrichment rounds: dictionaries,
    element levels and per-round counts bit-exact, coefficients to 1e-9."""
    g = synth.facies256(n=64, n_sub=4)
    S = api.partition(ctx, g)
    m_cap = 64 + 3 * 3 * 51
    D = api.init_lattice(ctx, g, [8, 8], m_cap=m_cap)
    od0 = O.init_dictionary(g, [8, 8], m_cap)
    tol = 1e-4 * (1 / 64) ** 2
    opts = api.EnetOpts(L1, L2, "f64", cd_sweeps=8)
    ro = api.RefineOpts(k_top=51, max_rounds=3, eps_tol=tol)
    beta, lvl, rounds, rs, stats = api.refine(ctx, S, D, opts, ro)
    torch.cuda.synchronize()
    Sn = O.partition(g)
    odr, bo, lvo, info = O.refine_batch(Sn, od0, L1, L2, k_top=51, max_rounds=3, m_max=1 << 30,
                                        eps_tol=tol)
    assert np.array_equal(_t(D.m), odr.m)
    assert np.array_equal(_t(lvl), lvo)
    assert np.array_equal(_t(rounds), info["rounds"])
    for s in range(D.n_sub):
        M = int(odr.m[s])
        assert np.array_equal(_t(D.c)[s, :M].ravel(), odr.c[s * m_cap * 2:(s * m_cap + M) * 2])
        assert np.array_equal(_t(D.sigma)[s, :M], odr.sigma[s * m_cap:s * m_cap + M])
        assert np.array_equal(_t(D.level)[s, :M], odr.level[s * m_cap:s * m_cap + M])
    ors = info["round_stats"]
    grs = _t(rs)
    assert np.array_equal(grs[..., 0], ors[..., 0])   # M per round
    assert np.array_equal(grs[..., 3], ors[..., 3])   # marked per round
    assert np.allclose(grs[..., 2], ors[..., 2], rtol=1e-8, atol=0)
    worst = _check_fit(Sn, odr, _t(beta), bo, L1, L2, 1e-9)
    print("max rel coefficient error", worst)


# ---------------------------------------------------------------- a10
def test_eval_matches_oracle(ctx):
    g = synth.circle64()
    D = api.init_lattice(ctx, g, [16, 16], m_cap=256)
    od = O.init_dictionary(g, [16, 16], 256)
    bnp, beta = _coefficients(od, 41)
    xq = synth.uniform_queries(2, 20000, seed=77, dtype=np.float64)
    xq[:3] = [[0.0, 0.0], [1.0, 1.0], [0.5, 0.5]]   # closed boundary and interior breakpoint
    xq_d = torch.as_tensor(xq, device="cuda")
    out64 = api.evaluate(ctx, g, D, beta, xq_d)
    out32 = api.evaluate(ctx, g, D, beta, xq_d.float())
    lin = api.evaluate(ctx, g, D, beta, xq_d, space=1)
    torch.cuda.synchronize()
    ref, nout = O.evaluate(O.grid_axis_coords(g), od, bnp.ravel(), xq)
    assert nout == 0
    assert np.max(np.abs(_t(out64) - ref)) <= 1e-12 * np.abs(ref).max()
    assert np.max(np.abs(_t(out32).astype(np.float64) - ref)) <= 2e-4 * max(1.0, np.abs(ref).max())
    assert np.allclose(_t(lin), 10.0 ** ref, rtol=1e-12)


def test_eval_of_a_fitted_field(ctx):
    """The fitted circle field evaluates to the oracle's own fitted field."""
    g = synth.circle64()
    S = api.partition(ctx, g)
    D = api.init_lattice(ctx, g, [16, 16], m_cap=256)
    beta, _ = api.fit(ctx, S, D, api.EnetOpts(L1, L2, "f64"))
    xq = synth.uniform_queries(2, 5000, seed=78, dtype=np.float64)
    out = api.evaluate(ctx, g, D, beta, torch.as_tensor(xq, device="cuda"))
    torch.cuda.synchronize()
    od = O.init_dictionary(g, [16, 16], 256)
    bo, sto, _ = O.fit_batch(O.partition(g), od, L1, L2, cd_sweeps=8)
    ref, _ = O.evaluate(O.grid_axis_coords(g), od, bo.ravel(), xq)
    assert np.max(np.abs(_t(out) - ref)) <= 1e-9 * np.abs(ref).max()


def test_eval_multifield_and_outside(ctx):
    grids = [synth.disc_field(5000 + f, n=32 * (2 + f)) for f in range(3)]
    Ds = [api.init_lattice(ctx, g, [8, 8], m_cap=64) for g in grids]
    ods = [O.init_dictionary(g, [8, 8], 64) for g in grids]
    bs = [_coefficients(od, 60 + f) for f, od in enumerate(ods)]
    Dall = api.Dictionary(sum(D.n_sub for D in Ds), 2, 64, torch.cat([D.m for D in Ds]),
                          torch.cat([D.c for D in Ds]), torch.cat([D.sigma for D in Ds]),
                          torch.cat([D.level for D in Ds]))
    ball = torch.cat([b[1] for b in bs])
    counts = [3000, 1, 2500]
    xs = [synth.uniform_queries(2, n, seed=90 + f, dtype=np.float64) for f, n in enumerate(counts)]
    xs[2][:2] = [[-0.1, 0.5], [0.5, 1.5]]            # outside the domain
    xq = torch.as_tensor(np.concatenate(xs), device="cuda")
    nout = torch.zeros(1, dtype=torch.int64, device="cuda")
    out = api.evaluate(ctx, grids, Dall, ball, xq, q_counts=counts, n_outside=nout)
    torch.cuda.synchronize()
    o = _t(out)
    assert int(nout.item()) == 2
    q0 = 0
    for f, g in enumerate(grids):
        ref, n_o = O.evaluate(O.grid_axis_coords(g), ods[f], bs[f][0].ravel(), xs[f])
        got = o[q0:q0 + counts[f]]
        assert np.array_equal(np.isnan(got), np.isnan(ref))
        ok = ~np.isnan(ref)
        assert np.max(np.abs(got[ok] - ref[ok]), initial=0.0) <= 1e-12 * max(1.0, np.abs(ref[ok]).max())
        q0 += counts[f]
