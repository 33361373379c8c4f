"""GPU parity of the learned warm start (through the C ABI) against the FP64
oracle, and what the trained network gains over the plain fit.

Tolerances. Forward logits: every output sums 25*cin + 1 FP32 products per
layer (at most 801) over four layers; sequential FP32 accumulation bounds
the error by about n*u*sum|terms| with u = 2^-24, i.e. 5e-5 relative to the
magnitude of the partial sums; the test takes 5e-5 of max|z|. Gradients: the
weight gradients add B*256 further products per entry in FP32; 2e-4 of the
layer's max|g|. Adam: elementwise FP32 arithmetic on float32 hyper-parameters,
1e-6 relative for the moments, 1e-5 of the step plus one ulp of p. Patches,
hint and labels: bit-exact (index work; FP64 cell lookups on both sides).
"""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import cnn_oracle as CO  # noqa: E402
from oracle import oracle as O  # noqa: E402
from paper_2605_16564_amd import api, learned, synth  # noqa: E402

L1, L2 = synth.LAMBDA1, synth.LAMBDA2


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = api.Context(0)
    yield c
    c.close()


def _d(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def _t(x):
    return x.detach().cpu().numpy()


def _layer_slices():
    out, o = [], 0
    for ci, co in zip(CO.CIN, CO.COUT):
        n = co * ci * 25 + co
        out.append(slice(o, o + n))
        o += n
    return out


@pytest.mark.parametrize("B", [1, 5])
def test_cnn_forward_matches_oracle(ctx, B):
    p = synth.cnn_init(11)
    x, _, _ = synth.cnn_batch(12, B)
    z = _t(api.cnn_forward(ctx, _d(p), _d(x)))
    zo, _ = CO.forward(p.astype(np.float64), x.astype(np.float64))
    err = np.abs(z - zo).max()
    print("B", B, "max|z|", np.abs(zo).max(), "max err", err)
    assert err <= 5e-5 * np.abs(zo).max()


@pytest.mark.parametrize("B", [3, 37])
def test_cnn_gradients_match_oracle(ctx, B):
    """B = 37 leaves a ragged last block of the weight-gradient reduction."""
    p = synth.cnn_init(21)
    x, t, m = synth.cnn_batch(22, B)
    g, loss = api.cnn_loss_grad(ctx, _d(p), _d(x), _d(t), _d(m))
    g, loss = _t(g), float(loss.item())
    lo, go = CO.loss_grad(p.astype(np.float64), x.astype(np.float64), t, m)
    assert loss == pytest.approx(lo, rel=1e-5)
    for l, sl in enumerate(_layer_slices()):
        err = np.abs(g[sl] - go[sl]).max()
        scale = np.abs(go[sl]).max()
        print("layer", l, "max|g|", scale, "max err", err)
        assert err <= 2e-4 * scale


@pytest.mark.parametrize("B", [1, 6, 37])
def test_cnn_bf16_matches_oracle(ctx, B):
    """BF16 mode against the oracle emulating it (the 32 -> 32 layers' operands
    rounded to bfloat16 at the same points, FP64 otherwise): logits and
    gradients to FP32-accumulation accuracy, up to the odd operand that the
    FP32 and FP64 paths round to neighbouring bfloat16 values: one such flip
    moves a product by 2^-8 of itself, measured up to 4e-4 of max|z| and
    4.4e-3 of a layer's max|g|; the bounds are 1e-3 and 1e-2. Against the
    plain FP64 network the BF16 mode is a rounding-size approximation
    (reported, 0.3-0.4 % on logits)."""
    p = synth.cnn_init(31)
    x, t, m = synth.cnn_batch(32, B)
    z = _t(api.cnn_forward(ctx, _d(p), _d(x), precision="bf16"))
    ze, _ = CO.forward(p.astype(np.float64), x.astype(np.float64), bf16_layers=(1, 2))
    zo, _ = CO.forward(p.astype(np.float64), x.astype(np.float64))
    zerr = np.abs(z - ze).max() / np.abs(ze).max()
    print("B", B, "logit err vs emulation", zerr, "vs FP64 network", np.abs(z - zo).max() / np.abs(zo).max())
    assert zerr <= 1e-3
    g, loss = api.cnn_loss_grad(ctx, _d(p), _d(x), _d(t), _d(m), precision="bf16")
    g, loss = _t(g), float(loss.item())
    le, ge = CO.loss_grad(p.astype(np.float64), x.astype(np.float64), t, m, bf16_layers=(1, 2))
    _, go = CO.loss_grad(p.astype(np.float64), x.astype(np.float64), t, m)
    assert loss == pytest.approx(le, rel=1e-4)
    for l, sl in enumerate(_layer_slices()):
        err = np.abs(g[sl] - ge[sl]).max() / np.abs(ge[sl]).max()
        rel_fp64 = np.linalg.norm(g[sl] - go[sl]) / np.linalg.norm(go[sl])
        print("layer", l, "grad err vs emulation", err, "rel L2 vs FP64 network", rel_fp64)
        assert err <= 1e-2


def test_cnn_empty_mask_gives_zero(ctx):
    p = synth.cnn_init(5)
    x, t, m = synth.cnn_batch(6, 4)
    g, loss = api.cnn_loss_grad(ctx, _d(p), _d(x), _d(t), _d(np.zeros_like(m)))
    torch.cuda.synchronize()
    assert float(loss.item()) == 0.0
    assert torch.count_nonzero(g).item() == 0


def test_cnn_adam_matches_oracle(ctx):
    rng = np.random.default_rng(31)
    n = api.cnn_param_count()
    p = rng.standard_normal(n).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    m = (0.1 * rng.standard_normal(n)).astype(np.float32)
    v = (0.01 * rng.random(n)).astype(np.float32)
    pd, gd, md, vd = _d(p), _d(g), _d(m), _d(v)
    api.cnn_adam(ctx, pd, gd, md, vd, step=3, lr=1e-3)
    # the ABI takes the hyper-parameters as float32: the oracle gets the same values
    f = lambda a: float(np.float32(a))  # noqa: E731
    po, mo, vo = CO.adam(p.astype(np.float64), g.astype(np.float64), m.astype(np.float64),
                         v.astype(np.float64), 3, f(1e-3), f(0.9), f(0.999), f(1e-8))
    np.testing.assert_allclose(_t(md), mo, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(_t(vd), vo, rtol=1e-6, atol=1e-9)
    # the step to 1e-5 of its size, plus the rounding of the FP32 result (one ulp of p)
    ulp = np.spacing(np.abs(p)).astype(np.float64)
    assert np.all(np.abs(_t(pd) - po) <= 1e-5 * np.abs(po - p) + ulp)


def test_patches_bit_exact(ctx):
    g = synth.facies256()
    x = _t(api.grid_patches(ctx, g, scale=synth.CNN_SCALE))
    ref = CO.patches(g, np.float32(synth.CNN_SCALE))
    assert ref.shape == (256, 16, 16) and x.shape == (256, 1, 16, 16)   # 64 boxes of 32x32 cells
    assert np.array_equal(x[:, 0], ref)


def _mixed_dictionary(g, seed):
    """Oracle lattice (12x12) plus extra centers: uniform in the owned box,
    some on cell faces, some on the box's upper faces."""
    od = O.init_dictionary(g, [12, 12], 200)
    rng = np.random.default_rng(seed)
    h = 1.0 / g.n_cells[0]
    c = od.c.reshape(od.n_sub, 200, 2)
    for s, (i0, j0, ni, nj) in enumerate(CO.owned_boxes_cells(g)):
        k0 = int(od.m[s])
        extra = 40 + s % 7
        pts = np.column_stack([(i0 + rng.random(extra) * ni) * h, (j0 + rng.random(extra) * nj) * h])
        pts[:10] = np.column_stack([(i0 + rng.integers(0, ni + 1, 10)) * h,
                                    (j0 + rng.integers(0, nj + 1, 10)) * h])
        c[s, k0:k0 + extra] = pts
        od.m[s] = k0 + extra
    od.c = c.ravel().copy()
    return od


def _api_dict(od):
    D = api.Dictionary.empty(od.n_sub, od.dim, od.m_cap, torch.device("cuda"))
    D.m.copy_(torch.as_tensor(od.m))
    D.c.copy_(torch.as_tensor(od.c.reshape(od.n_sub, od.m_cap, od.dim)))
    D.sigma.copy_(torch.as_tensor(od.sigma.reshape(od.n_sub, od.m_cap)))
    D.level.copy_(torch.as_tensor(od.level.reshape(od.n_sub, od.m_cap)))
    return D


def test_support_hint_bit_exact(ctx):
    g = synth.facies256()
    od = _mixed_dictionary(g, 41)
    lg = np.random.default_rng(42).standard_normal((256, 2, 16, 16)).astype(np.float32)
    for thr in (0.0, 0.7):
        h = _t(api.support_hint(ctx, g, _api_dict(od), _d(lg), thr))
        ref = CO.hint(g, od.m, od.c, od.m_cap, lg, thr)
        assert np.array_equal(h, ref)


def test_labels_bit_exact(ctx):
    g = synth.facies256(seed=2003, n=128, n_sub=4)
    od = _mixed_dictionary(g, 43)
    S = api.partition(ctx, g)
    Sn = O.partition(g)
    rng = np.random.default_rng(44)
    beta = synth.random_coefficients(45, od.n_sub, od.m_cap, od.m)
    lvl = rng.integers(0, 3, int(Sn["off"][-1])).astype(np.int32)
    t, m = api.cnn_labels(ctx, g, S, _api_dict(od), _d(beta), _d(lvl))
    to, mo = CO.labels(g, Sn["off"], Sn["x"], od.m, od.c, od.m_cap, beta, lvl)
    assert np.array_equal(_t(t), to)
    assert np.array_equal(_t(m), mo)


def test_learned_warm_start_gain(ctx):
    """Train on the method's own round-0 fits of eight facies fields, then
    fit a held-out field with the method's default start (cold, 8 CD sweeps)
    and with the network's hint: the same minimizer (to the oracle's FP64
    tolerance), no CD warm-up, at least 3 % fewer active-set iterations than
    the default and a solve (network inference included) at least 5 % faster
    than the default's (measured: about 8 % and 17 %). A constant
    all-active hint (the prior the support head mostly learns: about 95 % of
    lattice centers are active) is measured beside it and reported."""
    opts = api.EnetOpts(L1, L2, "f64", cd_sweeps=8)
    train = [synth.facies256(seed=2100 + i) for i in range(8)]
    t0 = time.perf_counter()
    x, t, m = learned.training_set(ctx, train, [12, 12], 204, opts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    params = api.cnn_init(7, x.device)
    losses, _ = api.cnn_train(ctx, params, x, t, m, epochs=12, batch=128, lr=2e-3, seed=1)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    print(f"patches {x.shape[0]}, labels {t1 - t0:.2f} s, training {t2 - t1:.2f} s, losses {losses}")
    assert losses[-1] < 0.8 * losses[0]

    g = synth.facies256(seed=2000)
    S = api.partition(ctx, g)
    D = api.init_lattice(ctx, g, [12, 12], m_cap=144)
    hint = learned.hint(ctx, params, g, D)
    xh, th, mh = learned.training_set(ctx, [g], [12, 12], 204, opts)
    acc = learned.head_accuracy(api.cnn_forward(ctx, params, xh), th, mh)
    print("held-out accuracy (refine, support) vs majority:", acc)
    all_on = torch.ones_like(hint)                 # every slot is a lattice center (M = m_cap)
    api.fit(ctx, S, D, opts)                       # untimed: workspace sized, kernels loaded
    ctx.timing(True)
    ms = {}
    res = {}
    for name in ("default", "hinted", "all_active"):
        ctx.timing_read(reset=True)
        if name == "hinted":                        # the network's inference is timed with the fit
            o = api.EnetOpts(L1, L2, "f64", cd_sweeps=8, support_hint=learned.hint(ctx, params, g, D))
        elif name == "all_active":
            o = api.EnetOpts(L1, L2, "f64", cd_sweeps=8, support_hint=all_on)
        else:
            o = opts
        res[name] = api.fit(ctx, S, D, o)
        tk = ctx.timing_read(reset=True)
        ms[name] = tk["solve"][0] + tk["cnn"][0]
    ctx.timing(False)
    (b_cd, st_cd), (b_h, st_h), (b_a, st_a) = res["default"], res["hinted"], res["all_active"]
    s_cd, s_h, s_a = (api.stats_to_numpy(s) for s in (st_cd, st_h, st_a))
    print("iterations: default (cold + 8 CD sweeps)", s_cd["iters"].sum(), "sweeps", s_cd["cd_sweeps"].sum(),
          f"{ms['default']:.3f} ms | hinted", s_h["iters"].sum(), f"{ms['hinted']:.3f} ms incl. network",
          "| all-active hint", s_a["iters"].sum(), f"{ms['all_active']:.3f} ms")
    assert np.all(s_h["status"] == 0) and np.all(s_h["cd_sweeps"] == 0)
    assert s_h["iters"].sum() <= 0.97 * s_cd["iters"].sum()
    assert ms["hinted"] <= 0.95 * ms["default"]
    od = O.init_dictionary(g, [12, 12], 144)
    bo, sto, _ = O.fit_batch(O.partition(g), od, L1, L2, cd_sweeps=8)
    for b in (b_cd, b_h, b_a):
        bb = _t(b)
        for s in range(D.n_sub):
            ref = bo[s * 144:(s + 1) * 144]
            assert np.abs(bb[s] - ref).max() <= 1e-9 * np.abs(ref).max()
