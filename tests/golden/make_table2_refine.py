"""Writes table2_refine5.txt: the FP64 oracle's adaptive refinement with the
structure of Table 2 (Exp. 1.1) on one subdomain: a 32 x 32 mesh of [0,1]^2,
one center per element (1,024, width h = 1/32), K_top = 204, eta = 1/2, five
enrichment rounds without a stopping test (eps_tol = 0), so the center counts
run 1024, 1636, 2248, 2860, 3472, 4084 as in the table; lambda1 = 4.59e-4,
lambda2 = 4.64e-6. The paper's Case 1/2 fields are not available: the field is
a three-facies field on the 32 x 32 mesh, generated as the facies workload
(seed 2010): a symmetric field such as the circle would make many indicator
values tie exactly, so that the marking could legitimately differ between
two correct computations. Reference of the GPU's large-dictionary test.

Per round: center count, support, largest indicator, marked count; then the
SHA-256 of the final dictionary (centers, widths, levels as little-endian
float64 / int32) and of the element levels, the L1 error of the surrogate over
the mesh (4 x 4 Gauss points per cell, log10 units) and the nonzero
coefficients in hexadecimal.

Calls only the oracle (and the seeded field generator). Run:
python tests/golden/make_table2_refine.py   (about an hour on one core)
"""
import hashlib
import sys
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

from oracle import oracle as O  # noqa: E402
from paper_2605_16564_amd import synth  # noqa: E402

M_CAP = 4096 + 64
OUT = Path(__file__).resolve().parent / "table2_refine5.txt"


def main():
    g = synth.facies256(seed=2010, n=32, n_sub=1)
    S = O.partition(g)
    D = O.init_dictionary(g, [32, 32], M_CAP)
    Dr, beta, lvl, info = O.refine_batch(S, D, synth.LAMBDA1, synth.LAMBDA2, k_top=204,
                                         max_rounds=5, m_max=1 << 30, eps_tol=0.0, cd_sweeps=8)
    M = int(Dr.m[0])
    c, sg, lv = Dr.c[:M * 2], Dr.sigma[:M], Dr.level[:M]
    b = beta[:M]
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(c, "<f8").tobytes())
    h.update(np.ascontiguousarray(sg, "<f8").tobytes())
    h.update(np.ascontiguousarray(lv, "<i4").tobytes())
    pts, wts, cell_of = synth.metric_points(g, 4)
    D1 = O.Dictionary(1, M, 2)
    D1.m[:] = M
    D1.c[:] = c
    D1.sigma[:] = sg
    v, nout = O.evaluate([np.array([0.0, 1.0]), np.array([0.0, 1.0])], D1, b, pts)
    assert nout == 0
    l1 = float(np.sum(wts * np.abs(v - g.y[cell_of])))
    rs = info["round_stats"][0]
    nr = int(info["rounds"][0])
    lines = ["# FP64 oracle, Table 2 structure on a 32 x 32 facies field; written by "
             "make_table2_refine.py (do not edit)",
             f"# m_cap {M_CAP}",
             f"status {int(info['status'][0])}",
             f"rounds {nr}"]
    for key, col in (("M", 0), ("support", 1), ("marked", 3)):
        lines.append(key + " " + " ".join(str(int(rs[r, col])) for r in range(nr)))
    lines.append("maxR " + " ".join(float(rs[r, 2]).hex() for r in range(nr)))
    lines.append(f"dict_sha256 {h.hexdigest()}")
    lines.append(f"elem_level_sha256 {hashlib.sha256(np.ascontiguousarray(lvl, '<i4').tobytes()).hexdigest()}")
    lines.append(f"l1 {l1.hex()}")
    nz = np.nonzero(b)[0]
    lines.append(f"nonzero {len(nz)}")
    for k in nz:
        lines.append(f"{k} {float(b[k]).hex()}")
    OUT.write_text("\n".join(lines) + "\n")
    print(f"M {M}, support {len(nz)}, L1 {l1:.6f}, counts {[int(rs[r, 0]) for r in range(nr)]}")


if __name__ == "__main__":
    main()
