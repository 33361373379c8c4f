"""Fits and refinements as one HIP graph launch per call (the batching
pattern: every round's launches for all subdomains captured together, with
the per-subdomain active flags the kernels read on the device) against the
same launches enqueued directly: identical bits. A cached graph is replayed
several times with the program's own eager work (resets of the dictionary
and outputs by torch kernels) and synchronizations between replays, and every
replay must equal the direct result; with kernel timing on the launches go
directly, with the same result and per-kernel timings."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2605_16564_amd import api, synth  # noqa: E402

L1, L2 = synth.LAMBDA1, synth.LAMBDA2


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = api.Context(0)
    yield c
    c.graphs(True)
    c.close()


def _state(D, beta, lvl, out):
    """Everything the call writes except the per-subdomain wall times (the
    last round-stats column and the stats' solve_us field)."""
    st = api.stats_to_numpy(out["stats"])
    fields = [torch.as_tensor(np.ascontiguousarray(st[f])) for f in st.dtype.names if f != "solve_us"]
    return [t.clone() for t in (D.m, D.c, D.sigma, D.level, beta, lvl, out["rounds"],
                                out["round_stats"][..., :6])] + fields


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_refine_graph_replays_match_direct_launches(ctx, prec):
    g = synth.facies256(n=64, n_sub=4)
    print("case graph refine facies 64x64", prec, flush=True)
    S = api.partition(ctx, g)
    m_cap = 64 + 3 * 3 * 51
    D = api.init_lattice(ctx, g, [8, 8], m_cap)
    D0 = D.clone()
    tol = 1e-4 * (1 / 64) ** 2
    o = api.EnetOpts(L1, L2, prec)
    ro = api.RefineOpts(k_top=51, max_rounds=3, eps_tol=tol)
    beta = torch.zeros((D.n_sub, m_cap), dtype=torch.float64, device="cuda")
    lvl = torch.zeros(int(S.off_host[-1]), dtype=torch.int32, device="cuda")
    out = dict(rounds=torch.zeros(D.n_sub, dtype=torch.int32, device="cuda"),
               round_stats=torch.zeros((D.n_sub, 4, 7), dtype=torch.float64, device="cuda"),
               stats=api.new_stats(D.n_sub, "cuda"))

    def reset():
        for a, b in ((D.m, D0.m), (D.c, D0.c), (D.sigma, D0.sigma), (D.level, D0.level)):
            a.copy_(b)
        beta.zero_(); lvl.zero_()
        for t in out.values():
            t.zero_()

    ctx.graphs(False)
    reset()
    api.refine(ctx, S, D, o, ro, beta=beta, elem_level=lvl, out=out, warm=False)
    torch.cuda.synchronize()
    ref = _state(D, beta, lvl, out)
    assert np.all(api.stats_to_numpy(out["stats"])["status"] == 0)
    assert int(out["rounds"].max()) == 4
    ctx.graphs(True)
    for rep in range(4):
        reset()
        torch.cuda.synchronize()
        api.refine(ctx, S, D, o, ro, beta=beta, elem_level=lvl, out=out, warm=False)
        ctx.sync()
        got = _state(D, beta, lvl, out)
        for i, (a, b) in enumerate(zip(ref, got)):
            assert torch.equal(a, b), (rep, i)
    # timing on: the launches go directly (per-kernel events), same bits
    ctx.timing(True)
    ctx.timing_read(reset=True)
    reset()
    api.refine(ctx, S, D, o, ro, beta=beta, elem_level=lvl, out=out, warm=False)
    tk = ctx.timing_read(reset=True)
    ctx.timing(False)
    got = _state(D, beta, lvl, out)
    for i, (a, b) in enumerate(zip(ref, got)):
        assert torch.equal(a, b), ("timed", i)
    print("timed graph:", {k: v for k, v in tk.items() if v[1]})
    assert tk["solve"][1] == 4 and tk["solve"][0] > 0.0
    assert tk["indicator"][1] == 4 and tk["mark"][1] == 4


def test_fit_graph_matches_direct_launches(ctx):
    g = synth.circle64()
    print("case graph fit circle64 replicas", flush=True)
    S1 = api.partition(ctx, g)
    D1 = api.init_lattice(ctx, g, [16, 16], 256)
    S, D = api.concat_samples([S1] * 16), api.concat_dicts([D1] * 16)
    ctx.graphs(False)
    b0, s0 = api.fit(ctx, S, D, api.EnetOpts(L1, L2, "f32"))
    torch.cuda.synchronize()
    n0 = api.stats_to_numpy(s0)
    ctx.graphs(True)
    beta = torch.zeros_like(b0)
    st = api.new_stats(D.n_sub, "cuda")
    for rep in range(3):
        beta.fill_(3.0)
        api.fit(ctx, S, D, api.EnetOpts(L1, L2, "f32"), beta=beta, stats=st, warm=False)
        ctx.sync()
        assert torch.equal(beta, b0), rep
        n1 = api.stats_to_numpy(st)
        for f in n0.dtype.names:
            if f != "solve_us":
                assert np.array_equal(n0[f], n1[f]), (rep, f)
