"""The two FP32/BF16 Gram paths (the normalized design stored in HBM and
read by the MFMA Gram tiles, or fused: Shepard denominators first, then each
Gram tile computing its design entries in LDS) give the same bits: fits and
refinements with either path forced are compared element by element, and the
tuned default picks one of them, records its choice in the JSON-lines cache
file and reproduces the same result."""
import json
import os

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
    c.gram_path("tuned")
    c.close()


def _fields(st):
    n = api.stats_to_numpy(st)
    return {f: n[f] for f in n.dtype.names if f != "solve_us"}


def _refine(ctx, g, lattice, k_top, rounds, prec, dim_cap=None):
    S = api.partition(ctx, g)
    m0 = int(np.prod(lattice))
    m_cap = dim_cap or m0 + rounds * 3 * k_top
    D = api.init_lattice(ctx, g, lattice, m_cap)
    o = api.EnetOpts(L1, L2, prec)
    ro = api.RefineOpts(k_top=k_top, max_rounds=rounds, eps_tol=0.0)
    beta, _, rounds, rstats, stats = api.refine(ctx, S, D, o, ro, warm=False)
    torch.cuda.synchronize()
    return D, beta, dict(rounds=rounds, round_stats=rstats, stats=stats)


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_fused_gram_fit_matches_materialized(ctx, prec):
    for name, g, lat, cap in (("facies 64x64, 4 subdomains", synth.facies256(n=64, n_sub=4), [8, 8], 64),
                              ("facies 96x96, 1 subdomain, 3 tiles", synth.facies256(n=96, n_sub=1), [12, 12], 160),
                              ("layered3d 24^3, 8 subdomains", synth.layered3d(24, 24, 24, (2, 2, 2)), [4, 4, 4], 64)):
        print("case gram paths fit", name, prec, flush=True)
        S = api.partition(ctx, g)
        D = api.init_lattice(ctx, g, lat, cap)
        res = {}
        for mode in ("materialized", "fused"):
            ctx.gram_path(mode)
            b, st = api.fit(ctx, S, D, api.EnetOpts(L1, L2, prec), warm=False)
            torch.cuda.synchronize()
            res[mode] = (b.clone(), _fields(st))
        print("status materialized", res["materialized"][1]["status"], "fused", res["fused"][1]["status"])
        assert torch.equal(res["materialized"][0], res["fused"][0]), name
        for f, v in res["materialized"][1].items():
            assert np.array_equal(v, res["fused"][1][f]), (name, f)


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_fused_gram_refine_matches_materialized(ctx, prec):
    g = synth.facies256(n=64, n_sub=4)
    print("case gram paths refine facies 64x64", prec, flush=True)
    got = {}
    for mode in ("materialized", "fused"):
        ctx.gram_path(mode)
        D, beta, out = _refine(ctx, g, [8, 8], 51, 3, prec)
        got[mode] = [t.clone() for t in (D.m, D.c, D.sigma, beta, out["rounds"], out["round_stats"][..., :6])]
        got[mode].append(_fields(out["stats"]))
    for i, (a, b) in enumerate(zip(got["materialized"][:-1], got["fused"][:-1])):
        assert torch.equal(a, b), i
    for f, v in got["materialized"][-1].items():
        assert np.array_equal(v, got["fused"][-1][f]), f
    assert int(got["fused"][4].max()) == 4


def test_tuner_records_choice_and_matches(ctx, tmp_path):
    path = tmp_path / "tune.jsonl"
    os.environ["PAM_TUNE_CACHE"] = str(path)
    try:
        # a bucket no other test uses: padded M 384 (m_cap 330), 2-D, FP32
        g = synth.facies256(n=80, n_sub=1)
        print("case gram tuner facies 80x80 m_cap 330", flush=True)
        S = api.partition(ctx, g)
        D = api.init_lattice(ctx, g, [10, 10], 330)
        res = {}
        for mode in ("tuned", "materialized", "fused"):
            ctx.gram_path(mode)
            b, st = api.fit(ctx, S, D, api.EnetOpts(L1, L2, "f32"), warm=False)
            torch.cuda.synchronize()
            res[mode] = b.clone()
        assert torch.equal(res["tuned"], res["materialized"])
        assert torch.equal(res["tuned"], res["fused"])
        lines = [json.loads(s) for s in path.read_text().splitlines() if s.strip()]
        mine = [e for e in lines if e["key"].startswith("gfx950/gram/f32/mpad384/")]
        print("tuner entries", mine)
        assert len(mine) == 1
        e = mine[0]
        assert e["path"] in ("fused", "materialized")
        assert e["ms_materialized"] > 0 and e["ms_fused"] > 0
        faster = "fused" if e["ms_fused"] < e["ms_materialized"] else "materialized"
        assert e["path"] == faster
    finally:
        del os.environ["PAM_TUNE_CACHE"]
