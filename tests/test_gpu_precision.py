"""Mixed precision against the FP64 oracle: FP32 / BF16 design and Gram on
MFMA, FP64 active-set solve and FP64 polish (conjugate gradients on the
final support with the FP64 design recomputed, preconditioned by the
inverse of the low-precision active block).

Gates: FP32 coefficients within 1e-5 of max|beta| per subdomain; BF16
coefficients reported; for both, the field's L1 error against the data
within 1e-3 of the oracle's, and refinement decisions of a three-round run
identical to the oracle's in FP32."""
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


def _cell_centers(g):
    n0, n1 = g.n_cells[0], g.n_cells[1]
    X, Y = np.meshgrid((np.arange(n0) + 0.5) / n0 * (g.hi[0] - g.lo[0]) + g.lo[0],
                       (np.arange(n1) + 0.5) / n1 * (g.hi[1] - g.lo[1]) + g.lo[1], indexing="xy")
    return np.column_stack([X.ravel(), Y.ravel()])


def _l1(field, g):
    """L1 error of a field sampled at the cell centers against the cell data."""
    cell = np.prod([(g.hi[a] - g.lo[a]) / g.n_cells[a] for a in range(2)])
    return float(np.abs(field - g.y).sum() * cell)


def _coef_err(beta_gpu, bo, m, m_cap):
    worst = 0.0
    for s in range(len(m)):
        ref = bo[s * m_cap:s * m_cap + int(m[s])]
        worst = max(worst, np.abs(beta_gpu[s, :int(m[s])] - ref).max() / np.abs(ref).max())
    return worst


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_low_precision_fit_matches_oracle(ctx, prec):
    g, lat, cap = synth.circle64(), [16, 16], 256
    S = api.partition(ctx, g)
    D = api.init_lattice(ctx, g, lat, m_cap=cap)
    beta, stats = api.fit(ctx, S, D, api.EnetOpts(L1, L2, prec))
    xc = _cell_centers(g)
    fld = api.evaluate(ctx, g, D, beta, torch.as_tensor(xc, device="cuda"))
    torch.cuda.synchronize()
    st = api.stats_to_numpy(stats)
    od = O.init_dictionary(g, lat, cap)
    bo, sto, _ = O.fit_batch(O.partition(g), od, L1, L2)
    ref_fld, _ = O.evaluate(O.grid_axis_coords(g), od, bo.ravel(), xc)
    err = _coef_err(_t(beta), bo, od.m, cap)
    l1g, l1o = _l1(_t(fld), g), _l1(ref_fld, g)
    print(prec, "coefficient error", err, "polish", st["polish"], "kkt", st["kkt"].max(),
          "L1 gpu", l1g, "oracle", l1o)
    assert np.all(st["status"] == 0)
    if prec == "f32":
        assert err <= 1e-5
    assert abs(l1g - l1o) <= 1e-3


def test_f32_refinement_matches_oracle(ctx):
    """Three rounds of Alg. 1 on a 64x64 facies field in FP32 mode: the
    same dictionaries and element levels as the FP64 oracle, coefficients
    within 1e-5."""
    g = synth.facies256(n=64, n_sub=4)
    S = api.partition(ctx, g)
    m_cap = 64 + 3 * 3 * 51
    D = api.init_lattice(ctx, g, [8, 8], m_cap=m_cap)
    tol = 1e-4 * (1 / 64) ** 2
    beta, lvl, rounds, rs, stats = api.refine(ctx, S, D, api.EnetOpts(L1, L2, "f32"),
                                              api.RefineOpts(k_top=51, max_rounds=3, eps_tol=tol))
    torch.cuda.synchronize()
    od0 = O.init_dictionary(g, [8, 8], m_cap)
    odr, bo, lvo, info = O.refine_batch(O.partition(g), od0, L1, L2, k_top=51, max_rounds=3,
                                        m_max=1 << 30, eps_tol=tol)
    st = api.stats_to_numpy(stats)
    print("polish", st["polish"], "kkt", st["kkt"].max())
    assert np.array_equal(_t(D.m), odr.m)
    assert np.array_equal(_t(lvl), lvo)
    err = _coef_err(_t(beta), bo, odr.m, m_cap)
    print("coefficient error", err)
    assert err <= 1e-5
