"""Full-size parity of the facies256 refinement's later rounds: the GPU's
three-round run of the whole 256 x 256 field (64 subdomains in the batched
launches, FP32 Gram + FP64 pass, workgroup teams as the benchmark runs them;
also with the FP64 and the BF16 Gram)
against the FP64 oracle's reference for four sampled subdomains, including
the two with the most solve work (tests/golden/facies256_refine3.txt, written
by tests/golden/make_facies256_refine.py from the oracle alone).

Gates (Alg. 1, Table 2's per-round structure): center, support and marked
counts of every round equal; the largest R_T of every round to 1e-6
relative; the final dictionary and the element levels bit-identical (SHA-256
of their bytes); coefficients within 1e-5 of max|beta| with the same nonzero
set outside degenerate coordinates (|beta| below 1e-9 max|beta|), 1e-9 with
the FP64 Gram; the L1 error of each subdomain's surrogate within 1e-3 of the
oracle's."""
import hashlib
from pathlib import Path

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2605_16564_amd import api, synth  # noqa: E402

GOLDEN = Path(__file__).resolve().parent / "golden" / "facies256_refine3.txt"


def _read_golden():
    subs, cur, m_cap = {}, None, None
    lines = [l for l in GOLDEN.read_text().splitlines() if l.strip()]
    i = 0
    while i < len(lines):
        l = lines[i]
        if l.startswith("# subdomains"):
            m_cap = int(l.split("m_cap")[1])
        elif l.startswith("sub "):
            cur = {}
            subs[int(l.split()[1])] = cur
        elif l.startswith("nonzero "):
            n = int(l.split()[1])
            idx, val = [], []
            for k in range(n):
                a, b = lines[i + 1 + k].split()
                idx.append(int(a)); val.append(float.fromhex(b))
            cur["nz"] = (np.array(idx), np.array(val))
            i += n
        elif not l.startswith("#"):
            key, *rest = l.split()
            cur[key] = rest
        i += 1
    return subs, m_cap


def _sha(*arrays):
    h = hashlib.sha256()
    for a, dt in arrays:
        h.update(np.ascontiguousarray(a, dt).tobytes())
    return h.hexdigest()


@pytest.mark.parametrize("prec,tol", [("f32", 1e-5), ("f64", 1e-9), ("bf16", 1e-5)])
def test_facies256_three_rounds_against_oracle_reference(prec, tol):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ref, m_cap = _read_golden()
    ctx = api.Context(0)
    g = synth.facies256()
    print("case facies256 full size, three rounds,", prec, "Gram, teams", flush=True)
    S = api.partition(ctx, g)
    D = api.init_lattice(ctx, g, [12, 12], m_cap)
    eps = 1e-4 * float(np.prod(g.cell_size))
    beta, lvl, rounds, rs, stats = api.refine(ctx, S, D, api.EnetOpts(synth.LAMBDA1, synth.LAMBDA2, prec),
                                              api.RefineOpts(k_top=204, max_rounds=3, eps_tol=eps))
    torch.cuda.synchronize()
    st = api.stats_to_numpy(stats)
    assert np.all(st["status"] == 0) and st["kkt"].max() < 1e-9
    c, sg, lv, b, el = (D.c.cpu().numpy(), D.sigma.cpu().numpy(), D.level.cpu().numpy(),
                        beta.cpu().numpy(), lvl.cpu().numpy())
    grs, nr, m = rs.cpu().numpy(), rounds.cpu().numpy(), D.m.cpu().numpy()
    boxes = O.grid_owned_boxes(g)
    for s, r in ref.items():
        n = int(r["rounds"][0])
        assert int(nr[s]) == n
        for key, col in (("M", 0), ("support", 1), ("marked", 3)):
            assert [int(v) for v in grs[s, :n, col]] == [int(v) for v in r[key]], (s, key)
        mr = np.array([float.fromhex(v) for v in r["maxR"]])
        assert np.allclose(grs[s, :n, 2], mr, rtol=1e-6, atol=0), s
        M = int(m[s])
        assert _sha((c[s, :M].ravel(), "<f8"), (sg[s, :M], "<f8"), (lv[s, :M], "<i4")) == r["dict_sha256"][0]
        a0, a1 = S.off_host[s], S.off_host[s + 1]
        assert _sha((el[a0:a1], "<i4")) == r["elem_level_sha256"][0]
        bo = np.zeros(M)
        bo[r["nz"][0]] = r["nz"][1]
        scale = np.abs(bo).max()
        err = np.abs(b[s, :M] - bo).max() / scale
        firm = np.abs(bo) > 1e-9 * scale
        gpu_nz = b[s, :M] != 0
        assert np.array_equal(gpu_nz[firm], np.ones(firm.sum(), bool)), s
        assert not np.any(gpu_nz & (bo == 0) & (np.abs(b[s, :M]) > 1e-9 * scale)), s
        # L1 of the subdomain's surrogate over its owned cells (as the reference)
        lo, hi = boxes[s]
        k0, k1 = s % 8, s // 8
        cells = np.array([ii + 256 * jj for jj in range(32 * k1, 32 * k1 + 32)
                          for ii in range(32 * k0, 32 * k0 + 32)])
        pts, wts, cell_of = synth.metric_points(g, 4, cells)
        D1 = O.Dictionary(1, M, 2)
        D1.m[:] = M
        D1.c[:] = c[s, :M].ravel()
        D1.sigma[:] = sg[s, :M]
        v, _ = O.evaluate([np.array([lo[0], hi[0]]), np.array([lo[1], hi[1]])], D1, b[s, :M], pts)
        l1 = float(np.sum(wts * np.abs(v - g.y[cell_of]))) / float(np.prod(hi - lo))
        l1_ref = float.fromhex(r["l1"][0])
        print(f"subdomain {s}: M {M}, support {int(gpu_nz.sum())}, coefficient error {err:.2e}, "
              f"L1 {l1:.6f} (oracle {l1_ref:.6f}), team {st['team'][s]}")
        assert err <= tol, (s, err)
        assert abs(l1 - l1_ref) <= 1e-3
    ctx.close()
