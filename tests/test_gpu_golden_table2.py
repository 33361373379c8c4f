"""The structure of Table 2 (Exp. 1.1) on the GPU: one 32 x 32 subdomain,
one center per element (1,024), K_top = 204, five enrichment rounds without
a stopping test, so the dictionary grows to 4,084 centers, past what the
solve's per-center vectors hold in LDS (they move to HBM beyond ~2,500).
Against the FP64 oracle's run of the same problem
(tests/golden/table2_refine5.txt, written by make_table2_refine.py from the
oracle alone; the paper's Case fields are not available, the field is a
three-facies field on the 32 x 32 mesh, seed 2010, without the symmetries
that would make indicator values tie).

Gates: the center counts of every round equal Table 2's 1024, 1636, 2248,
2860, 3472, 4084 and the oracle's, as do the supports and marked counts; the
largest R_T of every round to 1e-6 relative; the final dictionary and the
element levels bit-identical (SHA-256); coefficients within 1e-5 of
max|beta| with the FP32 and BF16 Gram, 1e-9 with the FP64 Gram, every coordinate the oracle holds above
1e-9 max|beta| nonzero on the GPU; the field's L1 error within 1e-3 of the
oracle's. The support counts are printed, not gated: with 4 centers per
sample and lambda2 = 4.64e-6 the smallest coefficients sit at the rounding
level of the solve."""
import hashlib
from pathlib import Path

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2605_16564_amd import api, synth  # noqa: E402

GOLDEN = Path(__file__).resolve().parent / "golden" / "table2_refine5.txt"
TABLE2 = Path(__file__).resolve().parent / "golden" / "table2_center_counts.txt"


def _read():
    rec, nz = {}, None
    lines = [l for l in GOLDEN.read_text().splitlines() if l.strip()]
    i = 0
    while i < len(lines):
        l = lines[i]
        if l.startswith("# m_cap"):
            rec["m_cap"] = int(l.split()[-1])
        elif l.startswith("nonzero "):
            n = int(l.split()[1])
            pairs = [lines[i + 1 + k].split() for k in range(n)]
            nz = (np.array([int(a) for a, _ in pairs]), np.array([float.fromhex(b) for _, b in pairs]))
            i += n
        elif not l.startswith("#"):
            key, *rest = l.split()
            rec[key] = rest
        i += 1
    rec["nz"] = nz
    return rec


@pytest.mark.parametrize("prec,tol", [("f32", 1e-5), ("f64", 1e-9), ("bf16", 1e-5)])
def test_table2_structure_to_4084_centers(prec, tol):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if "facies field" not in GOLDEN.read_text().splitlines()[0]:
        pytest.skip("the reference predates the asymmetric field; regenerate it with make_table2_refine.py")
    ref = _read()
    table2 = [int(l.split()[1]) for l in TABLE2.read_text().splitlines()
              if l.strip() and not l.startswith("#")]
    m_cap = ref["m_cap"]
    ctx = api.Context(0)
    g = synth.facies256(seed=2010, n=32, n_sub=1)
    print("case Table 2 structure: 32x32, 1024 -> 4084 centers,", prec, "Gram", flush=True)
    S = api.partition(ctx, g)
    D = api.init_lattice(ctx, g, [32, 32], m_cap)
    beta, lvl, rounds, rs, stats = api.refine(ctx, S, D, api.EnetOpts(synth.LAMBDA1, synth.LAMBDA2, prec),
                                              api.RefineOpts(k_top=204, max_rounds=5, eps_tol=0.0))
    torch.cuda.synchronize()
    st = api.stats_to_numpy(stats)
    grs = rs.cpu().numpy()[0]
    print("status", st["status"], "kkt", st["kkt"], "round solve ms", (grs[:, 6] / 1e3).round(1).tolist())
    assert st["status"][0] == 0 and st["kkt"][0] < 1e-9
    n = int(ref["rounds"][0])
    M = int(D.m.cpu().numpy()[0])
    counts = [int(v) for v in grs[:n, 0]]
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(D.c.cpu().numpy()[0, :M].ravel(), "<f8").tobytes())
    h.update(np.ascontiguousarray(D.sigma.cpu().numpy()[0, :M], "<f8").tobytes())
    h.update(np.ascontiguousarray(D.level.cpu().numpy()[0, :M], "<i4").tobytes())
    el = np.ascontiguousarray(lvl.cpu().numpy(), "<i4")
    same_dict = h.hexdigest() == ref["dict_sha256"][0]
    same_levels = hashlib.sha256(el.tobytes()).hexdigest() == ref["elem_level_sha256"][0]
    mr = np.array([float.fromhex(v) for v in ref["maxR"]])
    print("counts", counts, "supports", [int(v) for v in grs[:n, 1]], "oracle", ref["support"],
          "maxR rel diff", (np.abs(grs[:n, 2] - mr) / mr).max(), "dictionary equal", same_dict,
          "levels equal", same_levels)
    b = beta.cpu().numpy()[0, :M]
    bo = np.zeros(M)
    bo[ref["nz"][0]] = ref["nz"][1]
    scale = np.abs(bo).max()
    err = np.abs(b - bo).max() / scale
    firm = np.abs(bo) > 1e-9 * scale
    pts, wts, cell_of = synth.metric_points(g, 4)
    D1 = O.Dictionary(1, M, 2)
    D1.m[:] = M
    D1.c[:] = D.c.cpu().numpy()[0, :M].ravel()
    D1.sigma[:] = D.sigma.cpu().numpy()[0, :M]
    v, _ = O.evaluate([np.array([0.0, 1.0]), np.array([0.0, 1.0])], D1, b, pts)
    l1 = float(np.sum(wts * np.abs(v - g.y[cell_of])))
    l1_ref = float.fromhex(ref["l1"][0])
    print(f"M {M}, support {int((b != 0).sum())}, coefficient error {err:.2e}, firm coordinates "
          f"{int(firm.sum())} with {int(np.sum(b[firm] == 0))} zero on the GPU, L1 {l1:.6f} (oracle {l1_ref:.6f})")
    assert int(rounds.cpu().numpy()[0]) == n == 6
    assert counts == table2 == [int(v) for v in ref["M"]]
    assert [int(v) for v in grs[:n, 3]] == [int(v) for v in ref["marked"]]
    assert np.allclose(grs[:n, 2], mr, rtol=1e-6, atol=0)
    assert same_dict and same_levels
    assert np.all(b[firm] != 0)
    assert err <= tol
    assert abs(l1 - l1_ref) <= 1e-3
    ctx.close()
