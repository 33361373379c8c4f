"""The two-center configuration of the Sec. 4 theorem in two dimensions, an
interface at 30 degrees, through the C-ABI: the GPU fit of a 100 x 100 cell
step H(n . x) on [-1, 1]^2 with two centers at +-c n against the FP64
oracle's fit of the same samples, and the GPU evaluation of the fitted field
at the quadrature points of the rotated L1 integral against the oracle's
(FP64 to 1e-9 relative; FP32 Gram mode to the FP64 problem's 1e-6, since its
FP64 pass finishes the same FP64 problem)."""
import math

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


def _step_grid(th, n_cells=100):
    n = np.array([math.cos(th), math.sin(th)])
    g = (np.arange(n_cells) + 0.5) * (2.0 / n_cells) - 1.0
    X1, X2 = np.meshgrid(g, g, indexing="xy")   # axis 0 fastest in the flattened order
    y = ((X1 * n[0] + X2 * n[1]) > 0).astype(np.float64).ravel()
    grid = synth.Grid(2, [n_cells, n_cells], [-1.0, -1.0], [1.0, 1.0], [1, 1],
                      [synth.even_breaks(n_cells, 1), synth.even_breaks(n_cells, 1)], 0.0, y)
    xs = np.stack([X1.ravel(), X2.ravel()], axis=1)
    return grid, xs, y, n


def _rotated_points(th, k, n_t=200):
    """Quadrature points and weights of the rotated L1 integral over the
    square (t across the interface, u along it)."""
    ct, st = math.cos(th), math.sin(th)
    T, tmax = abs(ct - st), ct + st
    gx, gw = np.polynomial.legendre.leggauss(12)
    ux, uw = np.polynomial.legendre.leggauss(6)
    inner = np.unique(np.concatenate([np.geomspace(1e-3 / k, T, n_t // 2), [T]]))
    edges = np.concatenate([[0.0], inner, np.linspace(T, tmax, n_t // 4 + 1)[1:]])
    pts, wts, hs = [], [], []
    for side in (-1.0, 1.0):
        a, b = edges[:-1], edges[1:]
        t = side * ((0.5 * (a + b))[:, None] + 0.5 * (b - a)[:, None] * gx[None, :]).ravel()
        wt = (0.5 * (b - a)[:, None] * gw[None, :]).ravel()
        lo = np.maximum((t * ct - 1.0) / st, (-1.0 - t * st) / ct)
        hi = np.maximum(np.minimum((t * ct + 1.0) / st, (1.0 - t * st) / ct), lo)
        u = (0.5 * (lo + hi))[:, None] + 0.5 * (hi - lo)[:, None] * ux[None, :]
        wu = 0.5 * (hi - lo)[:, None] * uw[None, :]
        X = np.stack([t[:, None] * ct - u * st, t[:, None] * st + u * ct], axis=-1).reshape(-1, 2)
        pts.append(X)
        wts.append((wt[:, None] * wu).ravel())
        hs.append(np.repeat((t > 0).astype(float), u.shape[1]))
    X = np.clip(np.concatenate(pts), -1.0, 1.0)
    return X, np.concatenate(wts), np.concatenate(hs)


# FP32 mode needs every sample's Shepard denominator to stay a normal FP32
# number: the farthest cell from both centers is at r^2 = 1.87, so sigma >= 0.11
# (exp(-r^2 / 2 sigma^2) > 1.2e-38); below that the fit reports UNDERFLOW.
@pytest.mark.parametrize("prec,tol,sigma", [("f64", 1e-9, 0.04), ("f64", 1e-9, 0.09), ("f32", 1e-6, 0.12)])
def test_angled_two_center_fit_and_l1_match_oracle(ctx, prec, tol, sigma):
    th, c = math.radians(30.0), 0.3
    grid, xs, y, n = _step_grid(th)
    print("case 2-D angled step, 30 degrees, c 0.3, sigma", sigma, prec, flush=True)
    cen = np.stack([c * n, -c * n])
    S = api.partition(ctx, grid)
    D = api.Dictionary.empty(1, 2, 2, ctx.device)
    D.m[0] = 2
    D.c[0] = torch.as_tensor(cen, device="cuda")
    D.sigma[0] = sigma
    beta, st = api.fit(ctx, S, D, api.EnetOpts(0.0, 0.0, prec), warm=False)
    stats = api.stats_to_numpy(st)
    assert stats["status"][0] == 0
    b_gpu = beta[0, :2].cpu().numpy()
    b_ora, ost, _ = O.fit_one(xs, y, cen, np.array([sigma, sigma]), 0.0, 0.0)
    assert ost == 0
    err = np.max(np.abs(b_gpu - b_ora)) / np.max(np.abs(b_ora))
    print("coefficients", b_gpu, b_ora, "rel err", err)
    assert err < tol
    # the fitted field at the quadrature points of the rotated L1 integral
    k = 2.0 * c / sigma ** 2
    X, w, H = _rotated_points(th, k)
    v_gpu = api.evaluate(ctx, grid, D, beta, torch.as_tensor(X, device="cuda")).cpu().numpy()
    Dor = O.Dictionary(1, 2, 2)
    Dor.m[:] = 2
    Dor.c[:] = cen.ravel()
    Dor.sigma[:] = sigma
    axis = [np.array([-1.0, 1.0]), np.array([-1.0, 1.0])]
    v_ora, _ = O.evaluate(axis, Dor, b_ora, X)
    assert np.max(np.abs(v_gpu - v_ora)) < 10 * tol
    l1_gpu = float((w * np.abs(H - v_gpu)).sum())
    l1_ora = float((w * np.abs(H - v_ora)).sum())
    print("L1 gpu", l1_gpu, "oracle", l1_ora, "theorem per length", math.log(2) * sigma ** 2 / c)
    assert abs(l1_gpu - l1_ora) / l1_ora < 10 * tol
    ratio = l1_gpu / (2.0 / math.cos(th)) / (math.log(2) * sigma ** 2 / c)
    assert 0.5 < ratio < 2.0


def test_angled_step_fp32_underflow_is_reported(ctx):
    """With sigma = 0.04 the far cells' FP32 Gaussians underflow (exp(-584)):
    the FP32 mode reports PAM_ST_UNDERFLOW for the subdomain and returns zero
    coefficients, while the FP64 mode fits it."""
    th, c, sigma = math.radians(30.0), 0.3, 0.04
    grid, xs, y, n = _step_grid(th)
    print("case 2-D angled step, FP32 underflow, sigma 0.04", flush=True)
    S = api.partition(ctx, grid)
    D = api.Dictionary.empty(1, 2, 2, ctx.device)
    D.m[0] = 2
    D.c[0] = torch.as_tensor(np.stack([c * n, -c * n]), device="cuda")
    D.sigma[0] = sigma
    for prec, want in (("f32", 2), ("f64", 0)):
        beta, st = api.fit(ctx, S, D, api.EnetOpts(0.0, 0.0, prec), warm=False)
        assert api.stats_to_numpy(st)["status"][0] == want, prec
        if want:
            assert torch.count_nonzero(beta).item() == 0
