"""Writes facies256_refine3.txt: the FP64 oracle's three-round refinement of
sampled subdomains of the facies256 workload (256 x 256 three-facies field,
8 x 8 subdomains of 32 x 32 elements, 12 x 12 initial centers with sigma0 =
h_c, K_top = 204, eta = 1/2, eps_tol = 1e-4 |T|, lambda1 = 4.59e-4, lambda2 =
4.64e-6), the reference of the GPU's full-size refinement test.

Calls only the oracle (and the seeded field generator for its input). The
subdomains include the ones with the most solve work in the batched GPU run
(13 and 33). Per subdomain the file holds: the center count, support, largest
indicator and marked count of every round (Alg. 1, Table 2's structure); the
SHA-256 of the final dictionary (centers, widths and levels as little-endian
float64 / int32 bytes) and of the element levels, so that the GPU's
dictionary can be compared bit for bit; the L1 error of the subdomain's
surrogate over its owned cells (4 x 4 Gauss points per cell, log10 units);
and the nonzero coefficients in hexadecimal (exact).

Run: python tests/golden/make_facies256_refine.py  (about 7 minutes on 8 cores)
"""
import hashlib
import sys
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

from oracle import oracle as O  # noqa: E402
from paper_2605_16564_amd import synth  # noqa: E402

SUBS = [13, 33, 27, 50]
G0, K_TOP, ROUNDS = 12, 204, 3
M_CAP = G0 * G0 + ROUNDS * K_TOP * 3
OUT = Path(__file__).resolve().parent / "facies256_refine3.txt"


def dict_hash(c, sigma, level):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(c, "<f8").tobytes())
    h.update(np.ascontiguousarray(sigma, "<f8").tobytes())
    h.update(np.ascontiguousarray(level, "<i4").tobytes())
    return h.hexdigest()


def main():
    g = synth.facies256()
    S = O.partition(g)
    D = O.init_dictionary(g, [G0, G0], M_CAP)
    offs = [0]
    xs, ys, hs = [], [], []
    Ds = O.Dictionary(len(SUBS), M_CAP, 2)
    for i, s in enumerate(SUBS):
        a, b = S["off"][s], S["off"][s + 1]
        xs.append(S["x"][a:b]); ys.append(S["y"][a:b]); hs.append(S["h"][a:b])
        offs.append(offs[-1] + b - a)
        Ds.m[i] = D.m[s]
        Ds.c[i * M_CAP * 2:(i + 1) * M_CAP * 2] = D.c[s * M_CAP * 2:(s + 1) * M_CAP * 2]
        Ds.sigma[i * M_CAP:(i + 1) * M_CAP] = D.sigma[s * M_CAP:(s + 1) * M_CAP]
        Ds.level[i * M_CAP:(i + 1) * M_CAP] = D.level[s * M_CAP:(s + 1) * M_CAP]
    sub = dict(off=np.array(offs, np.int64), x=np.concatenate(xs), y=np.concatenate(ys),
               h=np.concatenate(hs))
    eps = 1e-4 * float(np.prod(g.cell_size))
    Dr, beta, lvl, info = O.refine_batch(sub, Ds, synth.LAMBDA1, synth.LAMBDA2, k_top=K_TOP,
                                         max_rounds=ROUNDS, m_max=1 << 30, eps_tol=eps)
    boxes = O.grid_owned_boxes(g)
    lines = ["# FP64 oracle, facies256, three enrichment rounds; written by "
             "make_facies256_refine.py (do not edit)",
             f"# subdomains {' '.join(map(str, SUBS))}; m_cap {M_CAP}"]
    for i, s in enumerate(SUBS):
        M = int(Dr.m[i])
        rs = info["round_stats"][i]
        nr = int(info["rounds"][i])
        c = Dr.c[i * M_CAP * 2:(i * M_CAP + M) * 2]
        sg = Dr.sigma[i * M_CAP:i * M_CAP + M]
        lv = Dr.level[i * M_CAP:i * M_CAP + M]
        el = lvl[sub["off"][i]:sub["off"][i + 1]]
        b = beta[i * M_CAP:i * M_CAP + M]
        lo, hi = boxes[s]
        k0, k1 = s % 8, s // 8
        cells = np.array([ii + 256 * jj for jj in range(32 * k1, 32 * k1 + 32)
                          for ii in range(32 * k0, 32 * k0 + 32)])
        pts, wts, cell_of = synth.metric_points(g, 4, cells)
        D1 = O.Dictionary(1, M, 2)
        D1.m[:] = M
        D1.c[:] = c
        D1.sigma[:] = sg
        v, nout = O.evaluate([np.array([lo[0], hi[0]]), np.array([lo[1], hi[1]])], D1, b, pts)
        assert nout == 0
        l1 = float(np.sum(wts * np.abs(v - g.y[cell_of]))) / float(np.prod(hi - lo))
        lines.append(f"sub {s}")
        lines.append(f"status {int(info['status'][i])}")
        lines.append(f"rounds {nr}")
        for key, col in (("M", 0), ("support", 1), ("marked", 3)):
            lines.append(key + " " + " ".join(str(int(rs[r, col])) for r in range(nr)))
        lines.append("maxR " + " ".join(float(rs[r, 2]).hex() for r in range(nr)))
        lines.append(f"dict_sha256 {dict_hash(c, sg, lv)}")
        lines.append(f"elem_level_sha256 {hashlib.sha256(np.ascontiguousarray(el, '<i4').tobytes()).hexdigest()}")
        lines.append(f"l1 {l1.hex()}")
        nz = np.nonzero(b)[0]
        lines.append(f"nonzero {len(nz)}")
        for k in nz:
            lines.append(f"{k} {float(b[k]).hex()}")
        print(f"subdomain {s}: M {M}, support {len(nz)}, L1 {l1:.6f}", flush=True)
    OUT.write_text("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
