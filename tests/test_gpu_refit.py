"""pam_refit_nonconverged through the C ABI: the subdomains whose stats read
PAM_ST_NOCONV are fitted again with the FP64 Gram from a cold start and get
exactly what a plain FP64 fit of the same dictionary gives them (the same
kernels, so the same bits); every other subdomain keeps its coefficients and
stats entry bit for bit. The FP64 fit itself is checked against the oracle
elsewhere; here its coefficients are also compared with the oracle's on the
refitted subdomains of the small case (Eq. elastic, Sec. 3.3)."""
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


def _no_time(st):
    n = api.stats_to_numpy(st)
    return {f: n[f].copy() for f in n.dtype.names if f != "solve_us"}


def _mark(stats, subs, status):
    """Write a status into the stats entries of the listed subdomains."""
    h = stats.cpu().numpy().copy()
    v = h.view(api.STATS_DTYPE)
    for s in subs:
        v["status"][s] = status
    stats.copy_(torch.as_tensor(h, device=stats.device))


def test_refit_marked_subdomains_only(ctx):
    g = synth.facies256(n=64, n_sub=4)
    print("case refit facies 64x64, 16 subdomains, FP32 fit, 5 marked", flush=True)
    S = api.partition(ctx, g)
    D = api.init_lattice(ctx, g, [8, 8], 64)
    beta, st = api.fit(ctx, S, D, api.EnetOpts(L1, L2, "f32"), warm=False)
    torch.cuda.synchronize()
    assert (api.stats_to_numpy(st)["status"] == 0).all()
    marked = [1, 4, 6, 11, 15]
    _mark(st, marked, 1)
    b0, s0 = beta.clone(), _no_time(st)
    api.refit_nonconverged(ctx, S, D, api.EnetOpts(L1, L2, "f32"), beta, st)
    b64, st64 = api.fit(ctx, S, D, api.EnetOpts(L1, L2, "f64"), warm=False)
    torch.cuda.synchronize()
    s1, s64 = _no_time(st), _no_time(st64)
    keep = [s for s in range(D.n_sub) if s not in marked]
    assert torch.equal(beta[keep], b0[keep])
    assert torch.equal(beta[marked], b64[marked])
    for f in s1:
        assert np.array_equal(s1[f][keep], s0[f][keep]), f
        assert np.array_equal(s1[f][marked], s64[f][marked]), f
    assert (s1["status"] == 0).all()
    # the refitted coefficients against the oracle
    off = S.off_host
    x = S.x.cpu().numpy()
    y = S.y.cpu().numpy()
    c = D.c.cpu().numpy()
    sg = D.sigma.cpu().numpy()
    m = D.m.cpu().numpy()
    for s in marked:
        xs, ys = x[off[s]:off[s + 1]], y[off[s]:off[s + 1]]
        bo, ost, _ = O.fit_one(xs, ys, c[s, :m[s]], sg[s, :m[s]], L1, L2)
        assert ost == 0
        err = np.abs(beta[s, :m[s]].cpu().numpy() - bo).max() / np.abs(bo).max()
        assert err < 1e-9, (s, err)


def test_refit_recovers_plain_basis_fp32_refinement(ctx):
    """The unnormalized basis refined in the FP32 mode on the full facies256
    field: the subdomains that end not converged are refitted with the FP64
    Gram on their final dictionaries; afterwards every subdomain is converged
    and carries what a plain FP64 fit of that dictionary gives."""
    wl = synth.workload("facies256")
    g = wl.grids[0]
    print("case refit facies256 plain basis FP32 refinement, 3 rounds", flush=True)
    S = api.partition(ctx, g)
    m_cap = wl.m0 + wl.max_rounds * 3 * wl.k_top
    D = api.init_lattice(ctx, g, wl.g, m_cap, wl.sigma_factor, basis="plain")
    o = api.EnetOpts(wl.lambda1, wl.lambda2, "f32")
    eps = wl.eps_tol_rel * float(np.prod(g.cell_size))
    ro = api.RefineOpts(k_top=wl.k_top, max_rounds=wl.max_rounds, eps_tol=eps, eta=wl.eta)
    beta, _, _, _, st = api.refine(ctx, S, D, o, ro, warm=False)
    torch.cuda.synchronize()
    s0 = _no_time(st)
    bad = np.flatnonzero(s0["status"] == 1)
    good = np.flatnonzero(s0["status"] == 0)
    print("not converged after the FP32 refinement:", len(bad), "of", D.n_sub)
    # 28 of 64 on this field with the current kernels; with none the refit
    # must leave everything as it was, which the checks below also cover
    assert len(good) + len(bad) == D.n_sub
    b0 = beta.clone()
    api.refit_nonconverged(ctx, S, D, o, beta, st)
    b64, st64 = api.fit(ctx, S, D, api.EnetOpts(wl.lambda1, wl.lambda2, "f64"), warm=False)
    torch.cuda.synchronize()
    s1, s64 = _no_time(st), _no_time(st64)
    print("not converged after the refit:", int((s1["status"] != 0).sum()))
    assert (s1["status"] == 0).all()
    assert torch.equal(beta[good], b0[good])
    assert torch.equal(beta[bad], b64[bad])
    for f in s1:
        assert np.array_equal(s1[f][good], s0[f][good]), f
        assert np.array_equal(s1[f][bad], s64[f][bad]), f


def test_refit_argument_errors(ctx):
    g = synth.facies256(n=32, n_sub=2)
    S = api.partition(ctx, g)
    D = api.init_lattice(ctx, g, [4, 4], 16)
    beta = torch.zeros((D.n_sub, D.m_cap), dtype=torch.float64, device="cuda")
    from paper_2605_16564_amd import native as N
    with pytest.raises(N.PamError):
        api.refit_nonconverged(ctx, S, D, api.EnetOpts(L1, L2, "f32"), beta, None)
