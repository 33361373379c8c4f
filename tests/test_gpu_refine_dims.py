"""Refinement (Alg. 1) in three and one dimensions on the GPU against the
FP64 oracle.

Three dimensions: a reduced layered field (12 x 10 x 17 cells, 2 x 2 x 3
subdomains of 150 or 180 elements), 3^3 initial centers, K_top =
floor(0.05 N_i) per subdomain as in the layered workload, three enrichment
rounds of 7 centers per marked element, in every precision mode; and the
first enrichment round of the full-size layered workload (60 x 220 x 85,
1,188 subdomains, 8^3 centers, FP32 Gram + FP64 pass) on sampled
subdomains. One dimension: the step of Example 1 refined for four rounds
(one center per marked element).

Gates: dictionaries (centers, widths, levels), element levels, rounds,
per-round center and marked counts bit-exact; the largest R_T of every round
to 1e-8 relative (FP64) / 1e-6 (FP32, BF16: computed from coefficients that
match to 1e-9 of their size); coefficients 1e-9 of max|beta| in FP64 and
1e-5 in FP32 / BF16 (after the FP64 pass)."""
import functools

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


def _compare_refinement(D, lvl, rounds, rs, beta, odr, lvo, info, bo, r_tol, b_tol):
    m_cap, d = odr.m_cap, odr.dim
    assert np.array_equal(_t(D.m), odr.m)
    assert np.array_equal(_t(lvl), lvo)
    assert np.array_equal(_t(rounds), info["rounds"])
    c, sg, lv, b = _t(D.c), _t(D.sigma), _t(D.level), _t(beta)
    worst = 0.0
    for s in range(odr.n_sub):
        M = int(odr.m[s])
        assert np.array_equal(c[s, :M].ravel(), odr.c[s * m_cap * d:(s * m_cap + M) * d]), s
        assert np.array_equal(sg[s, :M], odr.sigma[s * m_cap:s * m_cap + M]), s
        assert np.array_equal(lv[s, :M], odr.level[s * m_cap:s * m_cap + M]), s
        ref = bo[s * m_cap:s * m_cap + M]
        scale = max(np.abs(ref).max(), 1e-300)
        err = np.abs(b[s, :M] - ref).max() / scale
        worst = max(worst, err)
        assert err <= b_tol, (s, err)
        assert np.all(b[s, M:] == 0.0)
    grs, ors = _t(rs), info["round_stats"]
    assert np.array_equal(grs[..., 0], ors[..., 0])      # centers per round
    assert np.array_equal(grs[..., 3], ors[..., 3])      # marked per round
    assert np.allclose(grs[..., 2], ors[..., 2], rtol=r_tol, atol=0)
    return worst


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_refine_3d_matches_oracle(ctx, prec):
    g = synth.layered3d(nx=12, ny=10, nz=17, sub=(2, 2, 3))
    print("case layered 12x10x17 sub 2x2x3", prec, flush=True)
    S = api.partition(ctx, g)
    ktop = np.floor(0.05 * np.diff(S.off_host)).astype(np.int32)
    assert sorted(set(ktop)) == [7, 9]
    m_cap = 27 + 3 * 7 * int(ktop.max())
    D = api.init_lattice(ctx, g, [3, 3, 3], m_cap)
    ro = api.RefineOpts(k_top=0, k_top_sub=ktop, max_rounds=3, eps_tol=1e-4)
    beta, lvl, rounds, rs, stats = api.refine(ctx, S, D, api.EnetOpts(L1, L2, prec), ro)
    torch.cuda.synchronize()
    st = api.stats_to_numpy(stats)
    assert np.all(st["status"] == 0)
    od0 = O.init_dictionary(g, [3, 3, 3], m_cap)
    odr, bo, lvo, info = O.refine_batch(O.partition(g), od0, L1, L2, k_top=ktop, max_rounds=3,
                                        m_max=1 << 30, eps_tol=1e-4)
    assert np.all(info["status"] == 0)
    assert np.all(info["rounds"] == 4)            # every subdomain enriched three times
    assert np.all(odr.m > 27 + 7 * 7 * 2)
    tol_b, tol_r = (1e-9, 1e-8) if prec == "f64" else (1e-5, 1e-6)
    worst = _compare_refinement(D, lvl, rounds, rs, beta, odr, lvo, info, bo, tol_r, tol_b)
    print(prec, "3-D refinement max rel coefficient error", worst, "kkt", st["kkt"].max())


def test_refine_1d_matches_oracle(ctx):
    g = synth.step1d(64)
    print("case step1d 64", flush=True)
    S = api.partition(ctx, g)
    m_cap = 4 + 4 * 2
    D = api.init_lattice(ctx, g, [4], m_cap)
    tol = 1e-6 * (0.03125 / 64)
    ro = api.RefineOpts(k_top=2, max_rounds=4, eps_tol=tol)
    beta, lvl, rounds, rs, stats = api.refine(ctx, S, D, api.EnetOpts(L1, L2, "f64"), ro)
    torch.cuda.synchronize()
    assert np.all(api.stats_to_numpy(stats)["status"] == 0)
    od0 = O.init_dictionary(g, [4], m_cap)
    odr, bo, lvo, info = O.refine_batch(O.partition(g), od0, L1, L2, k_top=2, max_rounds=4,
                                        m_max=1 << 30, eps_tol=tol)
    assert info["rounds"][0] >= 3 and int(odr.m[0]) > 4
    worst = _compare_refinement(D, lvl, rounds, rs, beta, odr, lvo, info, bo, 1e-8, 1e-9)
    print("1-D refinement", [int(v) for v in info["round_stats"][0, :, 0]], "coef err", worst)


def _sub_problem(Sn, od, subs):
    offs = [0]
    xs, ys, hs = [], [], []
    for s in subs:
        a, b = Sn["off"][s], Sn["off"][s + 1]
        xs.append(Sn["x"][a:b]); ys.append(Sn["y"][a:b]); hs.append(Sn["h"][a:b])
        offs.append(offs[-1] + b - a)
    sub = dict(off=np.array(offs, np.int64), x=np.concatenate(xs), y=np.concatenate(ys),
               h=np.concatenate(hs))
    D = O.Dictionary(len(subs), od.m_cap, od.dim)
    for i, s in enumerate(subs):
        k, d = od.m_cap, od.dim
        D.m[i] = od.m[s]
        D.c[i * k * d:(i + 1) * k * d] = od.c[s * k * d:(s + 1) * k * d]
        D.sigma[i * k:(i + 1) * k] = od.sigma[s * k:(s + 1) * k]
        D.level[i * k:(i + 1) * k] = od.level[s * k:(s + 1) * k]
    return sub, D


_L3_SUBS = [100, 777]


@functools.lru_cache(maxsize=1)
def _layered3d_oracle_first_round(m_cap):
    """The oracle's first enrichment round of the sampled layered3d
    subdomains (computed once for the precisions below)."""
    g = synth.layered3d()
    Sn = O.partition(g)
    ktop = np.floor(0.05 * np.diff(Sn["off"])).astype(np.int32)
    sub, Ds = _sub_problem(Sn, O.init_dictionary(g, [8, 8, 8], m_cap), _L3_SUBS)
    out = O.refine_batch(sub, Ds, L1, L2, k_top=ktop[_L3_SUBS], max_rounds=1, m_max=1 << 30, eps_tol=1e-4)
    return Sn, sub, out


@pytest.mark.parametrize("prec,tol", [("f32", 1e-5), ("f64", 1e-9), ("bf16", 1e-5)])
def test_layered3d_first_enrichment_fullsize_sampled(ctx, prec, tol):
    """The full layered workload, one enrichment round in the batched launch
    (FP32 Gram + FP64 pass as the benchmark runs it; also the FP64 and the
    BF16 Gram): every fit certified; on two sampled subdomains the enriched
    dictionary, element levels, counts and coefficients against the
    oracle."""
    g = synth.layered3d()
    print("case layered3d full size, one enrichment round,", prec, "Gram", flush=True)
    S = api.partition(ctx, g)
    ktop = np.floor(0.05 * np.diff(S.off_host)).astype(np.int32)
    m_cap = 512 + 7 * int(ktop.max())
    D = api.init_lattice(ctx, g, [8, 8, 8], m_cap)
    ro = api.RefineOpts(k_top=0, k_top_sub=ktop, max_rounds=1, eps_tol=1e-4)
    beta, lvl, rounds, rs, stats = api.refine(ctx, S, D, api.EnetOpts(L1, L2, prec), ro)
    torch.cuda.synchronize()
    st = api.stats_to_numpy(stats)
    assert np.all(st["status"] == 0) and st["kkt"].max() < 1e-9
    subs = _L3_SUBS
    Sn, sub, (odr, bo, lvo, info) = _layered3d_oracle_first_round(m_cap)
    m_cap_ = m_cap
    c, sg, lv, b, lg = _t(D.c), _t(D.sigma), _t(D.level), _t(beta), _t(lvl)
    grs = _t(rs)
    worst = 0.0
    for i, s in enumerate(subs):
        M = int(odr.m[i])
        assert int(_t(D.m)[s]) == M and M == 512 + 7 * int(ktop[s])
        assert np.array_equal(c[s, :M].ravel(), odr.c[i * m_cap_ * 3:(i * m_cap_ + M) * 3])
        assert np.array_equal(sg[s, :M], odr.sigma[i * m_cap_:i * m_cap_ + M])
        assert np.array_equal(lv[s, :M], odr.level[i * m_cap_:i * m_cap_ + M])
        a0, a1 = Sn["off"][s], Sn["off"][s + 1]
        assert np.array_equal(lg[a0:a1], lvo[sub["off"][i]:sub["off"][i + 1]])
        assert np.array_equal(grs[s, :2, 0], info["round_stats"][i, :, 0])
        assert np.array_equal(grs[s, :2, 3], info["round_stats"][i, :, 3])
        ref = bo[i * m_cap_:i * m_cap_ + M]
        err = np.abs(b[s, :M] - ref).max() / np.abs(ref).max()
        worst = max(worst, err)
        assert err <= tol, (s, err)
    print("layered3d sampled first-enrichment coefficient error", prec, worst)
