#!/usr/bin/env python3
"""Benchmark of the PAM reconstruction hot path on one MI355X.

One step = the whole path on one batch of synthetic input, inputs resident in
HBM: sample gathering (a1), lattice dictionary (a2), Shepard design, MFMA
Gram, elastic-net solve, indicator, marking and enrichment for every
subdomain and round (a3-a9), then evaluation of the fitted field at the
4x4 Gauss points of every cell (a10, mesh transfer to a finer quadrature).

Default workload `facies256`: 256x256 three-facies field, 8x8 subdomains,
12x12 initial centers, up to 3 enrichment rounds (K_top = 204), FP32 design
and Gram with the FP64 pass. The metric is subdomain fits per second (one fit
= one subdomain-round); evaluation throughput and the field's L1 error are
reported beside it.

The learned warm start (on by default) is trained before the timed region on
fields of other seeds; inside the step the network's forward pass and the
hint map run before the first fit. Beside the timed step the record holds:
the comparator (the plain GPU fit: one launch per subdomain and kernel, every
refit from zero, no hint), the learned part's training throughput and gain,
the error of the GPU coefficients and field against the FP64 oracle on the
CPU sample, the oracle's own throughput on that sample, the per-subdomain
choice of the elastic-net parameters (alpha path + K-fold cross-validation:
its fits/s and the field it gives after refinement), and the interface
treatment on the fitted field (continuous reconstruction across subdomain
interfaces: its throughput and error beside the owner reconstruction's, and
the interface jump it removes).

Prints one JSON line. `--gpus N` with N > 1 is refused: this build runs on
one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))

# MI355X published peaks used for the roofline fractions.
PEAK_HBM_GBS = 8000.0
PEAK_MFMA = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}   # TFLOP/s, dense
# Vector ALU issue slots per second from the published vector peaks (an FMA
# is 2 flops in one slot): FP32 157.3 TFLOP/s, FP64 78.6 TFLOP/s. A FP32
# transcendental (v_exp_f32) takes 4 FP32 slots (measured at 1/4.4 of the FP32
# FMA slot rate on this chip).
SLOTS_F32 = 157.3e12 / 2.0
SLOTS_F64 = 78.6e12 / 2.0

# HBM bytes per launch of the dominant kernel from two rocprofv3 counter runs
# (FETCH_SIZE, WRITE_SIZE, scaled by a 1 GiB device copy), valid only for the
# kernel source they were taken on (sha256 prefix of its source files).
TRAFFIC = {("k_solve<float, true>", "facies256"): {"src": "bc19a27042e93647", "bytes_per_launch": 66.07e9}}
TRAFFIC_SOURCES = ["paper_2605_16564_amd/csrc/k_solve.hip", "paper_2605_16564_amd/csrc/pam_internal.h"]


def measured_traffic(kernel, workload):
    import hashlib
    rec = TRAFFIC.get((kernel, workload))
    if rec is None:
        return None
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        h.update((ROOT / f).read_bytes())
    return rec["bytes_per_launch"] if h.hexdigest()[:16] == rec["src"] else None


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="facies256")
    ap.add_argument("--precision", default=None, help="Gram precision override (f64|f32|bf16)")
    ap.add_argument("--cd-sweeps", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-subdomains", type=int, default=8)
    ap.add_argument("--cpu-sample-rounds", type=int, default=1)
    ap.add_argument("--no-learned", action="store_true", help="no learned warm start")
    ap.add_argument("--train-mosaics", type=int, default=12,
                    help="training fields: mosaics of 8x8 facies256 fields (16384 patches each)")
    ap.add_argument("--no-comparator", action="store_true")
    ap.add_argument("--no-paper-ablations", action="store_true",
                    help="skip the uniform-lattice sweep and the indicator-on-K run")
    ap.add_argument("--no-ablations", action="store_true",
                    help="skip the one-pattern-off runs (batching, precision, learned)")
    ap.add_argument("--no-continuity", action="store_true",
                    help="skip the interface-treatment measurements")
    ap.add_argument("--no-select", action="store_true",
                    help="skip the per-subdomain lambda selection measurement")
    ap.add_argument("--select-alphas", type=int, default=13,
                    help="path length (half-decade steps down to 1e-6 alpha_max by default)")
    ap.add_argument("--select-ratio", type=float, default=1e-6)
    ap.add_argument("--select-folds", type=int, default=5)
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other configurations (circle64 replicas, layered3d, multifield)")
    ap.add_argument("--no-darcy", action="store_true",
                    help="skip the Darcy consumer (pressure error of the reconstruction)")
    ap.add_argument("--blend", type=float, default=0.1,
                    help="interface band half-width as a fraction of the shorter neighbour")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run three device copies of 1 GiB (scale for the HBM byte counters)")
    return ap.parse_args()


def cpu_baseline(grid, wl, n_sub_sample: int, rounds: int):
    """Time the FP64 CPU oracle on a bounded sample of the same workload:
    Alg. 1 with `rounds` enrichment rounds on `n_sub_sample` interior
    subdomains, one OpenMP thread per subdomain (the full three rounds take
    about 290 s per subdomain on one core). Returns the JSON record and the
    oracle's results (first subdomain, dictionary, coefficients)."""
    from oracle import oracle as O
    S = O.partition(grid)
    n = min(n_sub_sample, len(S["off"]) - 1)
    # an interior band of subdomains (row 3 of the 8x8 grid) with all facies
    first = min(3 * grid.n_sub[0], len(S["off"]) - 1 - n)
    j0, j1 = S["off"][first], S["off"][first + n]
    sub = dict(off=S["off"][first:first + n + 1] - j0, x=S["x"][j0:j1], y=S["y"][j0:j1],
               h=S["h"][j0:j1])
    D = O.init_dictionary(grid, wl.g, wl.m0 + wl.max_rounds * wl.k_top * (2 ** grid.dim - 1))
    Ds = O.Dictionary(n, D.m_cap, grid.dim)
    Ds.m = D.m[first:first + n].copy()
    Ds.c = D.c[first * D.m_cap * grid.dim:(first + n) * D.m_cap * grid.dim].copy()
    Ds.sigma = D.sigma[first * D.m_cap:(first + n) * D.m_cap].copy()
    Ds.level = D.level[first * D.m_cap:(first + n) * D.m_cap].copy()
    eps = wl.eps_tol_rel * float(np.prod(grid.cell_size))
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    Do, bo, _, info = O.refine_batch(sub, Ds, wl.lambda1, wl.lambda2, k_top=wl.k_top,
                                     max_rounds=rounds, m_max=1 << 30, eps_tol=eps)
    dt = time.perf_counter() - t0
    fits = int(info["rounds"].sum())
    rec = {"value": fits / dt, "unit": "subdomain fits/s", "cores": min(threads, n),
           "kind": "oracle",
           "sample": f"Alg. 1 with {rounds} of the {wl.max_rounds} enrichment rounds on {n} of "
                     f"{len(S['off']) - 1} subdomains ({fits} fits up to "
                     f"M={wl.m0 + rounds * wl.k_top * (2 ** grid.dim - 1)}, {dt:.1f} s, FP64, "
                     f"one OpenMP thread per subdomain); later rounds are slower per fit"}
    return rec, (first, n, sub, Do, bo, rounds)


def local_field(c, sigma, beta, x):
    """Normalized expansion sum_m beta_m phi_m(x) / sum_m phi_m(x) (FP64)."""
    d2 = ((x[:, None, :] - c[None, :, :]) ** 2).sum(-1)
    phi = np.exp(-d2 / (2.0 * sigma[None, :] ** 2))
    return (phi @ beta) / phi.sum(1)


def oracle_check(ctx, api, grid, wl, prec, opts, sample):
    """Same rounds on the GPU: dictionaries, coefficients and the field's L1
    error on the sample's owned cells against the oracle's."""
    import torch
    first, n, sub, Do, bo, rounds = sample
    S = api.partition(ctx, grid)
    D = api.init_lattice(ctx, grid, wl.g, Do.m_cap, wl.sigma_factor)
    eps = wl.eps_tol_rel * float(np.prod(grid.cell_size))
    beta, _, _, _, _ = api.refine(ctx, S, D, opts, api.RefineOpts(k_top=wl.k_top, max_rounds=rounds,
                                                                  eps_tol=eps, eta=wl.eta))
    torch.cuda.synchronize()
    m = D.m.cpu().numpy()[first:first + n]
    c = D.c.cpu().numpy()[first:first + n]
    sg = D.sigma.cpu().numpy()[first:first + n]
    b = beta.cpu().numpy()[first:first + n]
    same_dict = bool(np.array_equal(m, Do.m))
    err, l1g, l1o = 0.0, 0.0, 0.0
    cell = float(np.prod(grid.cell_size))
    for s in range(n):
        M = int(Do.m[s])
        ref = bo[s * Do.m_cap:s * Do.m_cap + M]
        co = Do.c[s * Do.m_cap * grid.dim:(s * Do.m_cap + M) * grid.dim].reshape(M, grid.dim)
        so = Do.sigma[s * Do.m_cap:s * Do.m_cap + M]
        same_dict &= bool(np.array_equal(c[s, :M], co) and np.array_equal(sg[s, :M], so))
        err = max(err, float(np.abs(b[s, :M] - ref).max() / np.abs(ref).max()))
        xs = sub["x"][sub["off"][s]:sub["off"][s + 1]]
        ys = sub["y"][sub["off"][s]:sub["off"][s + 1]]
        l1g += float(np.abs(local_field(c[s, :M], sg[s, :M], b[s, :M], xs) - ys).sum()) * cell
        l1o += float(np.abs(local_field(co, so, ref, xs) - ys).sum()) * cell
    return {"coef_rel_err_max": err, "gate_coef": 1e-5 if prec == "f32" else None,
            "field_l1_gpu": l1g, "field_l1_oracle": l1o, "gate_l1": 1e-3,
            "dictionaries_equal": same_dict,
            "sample": f"{n} subdomains from {first}, {rounds} enrichment round(s), "
                      "L1 over their samples' cells"}


def train_learned(ctx, api, wl, prec, n_mosaics):
    """Train the warm-start network (BF16 MFMA path) on the method's own fits
    of fields of other seeds, outside the timed region: n_mosaics mosaics of
    8 x 8 facies256 fields, 16384 patches each; returns (params, record)."""
    import torch
    from paper_2605_16564_amd import learned, synth
    opts = api.EnetOpts(wl.lambda1, wl.lambda2, prec)
    grids = [synth.facies_mosaic(seed=10000 + 64 * i) for i in range(n_mosaics)]
    t0 = time.perf_counter()
    x, t, m = learned.training_set(ctx, grids, wl.g, wl.k_top, opts, wl.eps_tol_rel)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    params = api.cnn_init(7, x.device)
    epochs, batch = 4, 1024
    ctx.timing(True)
    ctx.timing_read(reset=True)
    losses, _ = api.cnn_train(ctx, params, x, t, m, epochs=epochs, batch=batch, lr=2e-3, seed=1,
                              precision="bf16")
    tk = ctx.timing_read(reset=True)
    ctx.timing(False)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    n = int(x.shape[0])
    # fwd 27.4 MFLOP per patch (2 * 256 pixels * sum of cin*cout*25); fwd+bwd ~3x
    f_fwd = 2.0 * 256 * 25 * (1 * 32 + 32 * 32 + 32 * 32 + 32 * 2)
    flops = 3.0 * f_fwd * n * epochs
    cnn_ms = tk["cnn"][0]
    peak = 2500.0          # dense BF16 MFMA, TFLOP/s (the thin layers run on FP32 vector ALUs)
    ach = flops / (cnn_ms / 1e3) / 1e12
    rec = {"train_patches": n, "epochs": epochs, "batch": batch, "precision": "bf16",
           "loss_first": losses[0], "loss_last": losses[-1], "labels_s": t1 - t0, "train_s": t2 - t1,
           "train_patches_per_s": n * epochs / (t2 - t1),
           "roofline": {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                        "frac": ach / peak, "traffic": None,
                        "kernel": "network training (k_conv32_mfma, k_wgrad32_mfma, thin layers)"}}
    return params, rec


def learned_gain(ctx, api, grid, wl, prec, params):
    """Cold first-round fits of the bench field with and without the hint."""
    import torch
    from paper_2605_16564_amd import learned
    S = api.partition(ctx, grid)
    D = api.init_lattice(ctx, grid, wl.g, wl.m0, wl.sigma_factor)
    out = {}
    for name, hinted in (("cd_warmup", False), ("hinted", True)):
        ctx.timing(True)
        ctx.timing_read(reset=True)
        hint = learned.hint(ctx, params, grid, D, precision="bf16") if hinted else None
        beta, st = api.fit(ctx, S, D, api.EnetOpts(wl.lambda1, wl.lambda2, prec, support_hint=hint))
        tk = ctx.timing_read(reset=True)
        ctx.timing(False)
        s = api.stats_to_numpy(st)
        out[name] = {"solve_ms": tk["solve"][0], "cnn_ms": tk["cnn"][0],
                     "iters": int(s["iters"].sum()), "cd_sweeps": int(s["cd_sweeps"].sum()),
                     "beta": beta}
    b0, b1 = out["cd_warmup"].pop("beta"), out["hinted"].pop("beta")
    out["coef_rel_diff"] = float((b0 - b1).abs().max().item() / b0.abs().max().item())
    x, t, m = learned.training_set(ctx, [grid], wl.g, wl.k_top, api.EnetOpts(wl.lambda1, wl.lambda2, prec),
                                   wl.eps_tol_rel)
    acc = learned.head_accuracy(api.cnn_forward(ctx, params, x, "bf16"), t, m)
    out["held_out_accuracy"] = {"refine": acc[0][0], "refine_majority": acc[0][1],
                                "support": acc[1][0], "support_majority": acc[1][1]}
    return out


def lambda_selection(ctx, api, grid, wl, prec, m_cap, eps, xq, w_d, ycell, area, n_alpha, k_folds,
                     ratio, reps=2):
    """Per-subdomain parameters on the workload's initial lattice: the path
    timed with HIP events (fits = n_sub * k_folds * n_alpha), then a full
    refinement with the chosen parameters against the fixed pair."""
    import torch
    cell_y = torch.as_tensor(grid.y, dtype=torch.float64, device="cuda")
    S = api.partition(ctx, grid, cell_y)
    D0 = api.init_lattice(ctx, grid, wl.g, wl.m0, wl.sigma_factor)   # the initial lattice only
    o = api.EnetOpts(0.0, 0.0, prec)
    out = api.select_lambda(ctx, S, D0, o, n_alpha=n_alpha, k_folds=k_folds, alpha_min_ratio=ratio)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = api.select_lambda(ctx, S, D0, o, n_alpha=n_alpha, k_folds=k_folds,
                                alpha_min_ratio=ratio)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    fits = D0.n_sub * k_folds * n_alpha
    res = {"n_alpha": n_alpha, "k_folds": k_folds, "alpha_min_ratio": ratio, "l1_ratio": 0.99,
           "fits": fits, "ms": dt * 1e3, "fits_per_s": fits / dt,
           "n_failed": int(out["n_failed"].sum().item())}
    best = out["best"].cpu().numpy()
    res["chosen_index_histogram"] = np.bincount(best, minlength=n_alpha).tolist()
    l1 = out["lambda1"].cpu().numpy()
    res["lambda1_chosen"] = {"min": float(l1.min()), "median": float(np.median(l1)),
                             "max": float(l1.max())}
    fields = {}
    for name, kw in (("fixed_pair", dict(lambda1=wl.lambda1, lambda2=wl.lambda2)),
                     ("selected", dict(lambda1=0.0, lambda2=0.0, lambda1_sub=out["lambda1"],
                                       lambda2_sub=out["lambda2"]))):
        D = api.init_lattice(ctx, grid, wl.g, m_cap, wl.sigma_factor)
        ro = api.RefineOpts(k_top=wl.k_top, max_rounds=wl.max_rounds, eps_tol=eps, eta=wl.eta)
        beta, lvl, rounds, rs, st = api.refine(ctx, S, D, api.EnetOpts(precision=prec, **kw), ro)
        f = api.evaluate(ctx, grid, D, beta, xq)
        fields[name] = {"field_l1_log10": float((w_d * (f.double() - ycell).abs()).sum().item()) / area,
                        "centers_mean": float(D.m.double().mean().item()),
                        "support_mean": float(api.stats_to_numpy(st)["support"].mean())}
    res["refined_field"] = fields
    return res


def darcy(ctx, api, grid, D, beta, blend):
    """Pressure experiment of Exp. 1 on the fitted field: P1 elements on the
    data grid, K = 10^K* at the triangle centroids (owner and continuous
    reconstructions) against the data's own coefficient; CG timed with HIP
    events (one launch group per solve)."""
    import torch
    if grid.dim != 2:
        return None
    o = api.DarcyOpts(grid.n_cells[0], grid.n_cells[1], grid.lo[:2], grid.hi[:2], tol=1e-10)
    k_true = api.darcy_k_from_cells(ctx, grid, o)
    k_own = api.darcy_k_from_reconstruction(ctx, grid, D, beta, o)
    k_blend = api.darcy_k_from_reconstruction(ctx, grid, D, beta, o, blend=blend)
    torch.cuda.synchronize()
    ctx.timing(True)
    ctx.timing_read(reset=True)
    res = {"mesh": [o.n0, o.n1], "nodes": (o.n0 + 1) * (o.n1 + 1), "tol": o.tol}
    p = {}
    for name, k in (("true", k_true), ("owner", k_own), ("continuous", k_blend)):
        p[name], it, rel = api.darcy_solve(ctx, o, k)
        tk = ctx.timing_read(reset=True)["darcy"]
        res[name] = {"iterations": it, "rel_residual": rel, "ms": tk[0]}
    ctx.timing(False)
    res["E_p_owner"] = api.darcy_error(ctx, o, p["true"], p["owner"])
    res["E_p_continuous"] = api.darcy_error(ctx, o, p["true"], p["continuous"])
    # CG bytes per iteration: stencil pass (d, two edge arrays, q), update
    # (x, d, r, q, diag read; x, r, z written), direction (z, d read; d written)
    n = res["nodes"]
    it = res["true"]["iterations"]
    bytes_it = 8.0 * n * 15
    ach = bytes_it * it / (res["true"]["ms"] / 1e3) / 1e9
    res["roofline"] = {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                       "frac": ach / PEAK_HBM_GBS, "bytes_per_iteration": bytes_it,
                       "note": "three launches per iteration on a 66k-node mesh: launch latency, "
                               "not HBM, sets the time"}
    return res


def sub_problem(api, S, D, lo, hi):
    """Samples and dictionary of subdomains lo..hi-1 (device slices)."""
    import torch
    a, b = int(S.off_host[lo]), int(S.off_host[hi])
    off_h = S.off_host[lo:hi + 1] - a
    n_max = int(np.diff(off_h).max()) if hi > lo else 0
    Ss = api.Samples(S.dim, hi - lo, n_max, torch.as_tensor(off_h, device=S.x.device), off_h,
                     S.x[a:b], S.y[a:b], S.h[a:b])
    Ds = api.Dictionary(hi - lo, D.dim, D.m_cap, D.m[lo:hi].clone(), D.c[lo:hi].clone(),
                        D.sigma[lo:hi].clone(), D.level[lo:hi].clone(), D.basis)
    return Ss, Ds


def other_configs(ctx, api, synth, progress):
    """The other configurations as single timed runs (wall clock around
    synchronized calls, kernel split from HIP events): circle64 as 1,024
    replicas (4,096 FP64 fits), layered3d (1,188 subdomains, FP32 Gram + FP64
    pass, three enrichment rounds; the same with the BF16 Gram beside it),
    multifield (5,820 FP32 fits, then 6.4e7 FP32 query evaluations)."""
    import torch
    L1, L2 = synth.LAMBDA1, synth.LAMBDA2
    out = {}

    def timed(fn):
        fn()                                   # untimed: kernels loaded, workspace sized
        torch.cuda.synchronize()
        ctx.timing(True)
        ctx.timing_read(reset=True)
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        tk = ctx.timing_read(reset=True)
        ctx.timing(False)
        return r, dt, {k: v[0] for k, v in tk.items() if v[1] > 0}

    g = synth.circle64()
    S1 = api.partition(ctx, g)
    D1 = api.init_lattice(ctx, g, [16, 16], 256)
    reps = 1024
    S, D = api.concat_samples([S1] * reps), api.concat_dicts([D1] * reps)
    (beta, st), dt, tk = timed(lambda: api.fit(ctx, S, D, api.EnetOpts(L1, L2, "f64")))
    stn = api.stats_to_numpy(st)
    out["circle64_x1024"] = {"fits": D.n_sub, "s": dt, "fits_per_s": D.n_sub / dt, "dtype": "f64",
                             "status_ok": bool(np.all(stn["status"] == 0)),
                             "kkt_max": float(stn["kkt"].max()), "kernel_ms": tk}
    progress("circle64 replicas done")

    g3 = synth.layered3d()
    S3 = api.partition(ctx, g3)
    ktop = np.floor(0.05 * np.diff(S3.off_host)).astype(np.int32)
    m_cap = 512 + 3 * int(ktop.max()) * 7

    def run3(prec):
        D3 = api.init_lattice(ctx, g3, [8, 8, 8], m_cap)
        r = api.refine(ctx, S3, D3, api.EnetOpts(L1, L2, prec),
                       api.RefineOpts(k_top=0, k_top_sub=ktop, max_rounds=3, eps_tol=1e-4))
        return D3, r
    for key, prec in (("layered3d", "f32"), ("layered3d_bf16", "bf16")):
        (D3, (b3, lvl3, rounds3, rs3, st3)), dt, tk = timed(lambda: run3(prec))
        stn = api.stats_to_numpy(st3)
        fits = int(rounds3.sum().item())
        out[key] = {"subdomains": D3.n_sub, "fits": fits, "s": dt, "fits_per_s": fits / dt,
                    "dtype": prec, "centers_final_mean": float(D3.m.double().mean().item()),
                    "status_ok": bool(np.all(stn["status"] == 0)),
                    "kkt_max": float(stn["kkt"].max()), "kernel_ms": tk}
        progress(key + " done")

    grids = synth.multifield()
    parts = [api.partition(ctx, gg) for gg in grids]
    dicts = [api.init_lattice(ctx, gg, [16, 16], 256) for gg in grids]
    S5, D5 = api.concat_samples(parts), api.concat_dicts(dicts)
    (b5, st5), dt, tk = timed(lambda: api.fit(ctx, S5, D5, api.EnetOpts(L1, L2, "f32")))
    stn = api.stats_to_numpy(st5)
    Q = 1_000_000
    xs = np.concatenate([synth.uniform_queries(2, Q, seed=5100 + f) for f in range(len(grids))])
    xq = torch.as_tensor(xs, device="cuda")
    o5, dte, tke = timed(lambda: api.evaluate(ctx, grids, D5, b5, xq, q_counts=[Q] * len(grids)))
    out["multifield"] = {"fields": len(grids), "subdomains": D5.n_sub, "fit_s": dt,
                         "fits_per_s": D5.n_sub / dt, "queries": Q * len(grids), "eval_s": dte,
                         "query_evals_per_s": Q * len(grids) / dte, "dtype": "f32",
                         "status_ok": bool(np.all(stn["status"] == 0)),
                         "kkt_max": float(stn["kkt"].max()), "fit_kernel_ms": tk,
                         "eval_kernel_ms": tke}
    progress("multifield done")
    return out


def paper_ablations(ctx, api, grid, wl, prec, m_cap, eps, xq, w_d, ycell, area, progress):
    """The comparisons the paper makes with the method's own parts: uniform
    lattices of growing size without refinement (Table 1, Example 2) against
    the adaptive result, and the refinement indicator measured on K itself
    (Alg. 1 literal) instead of log10 K."""
    import torch
    cell_y = torch.as_tensor(grid.y, dtype=torch.float64, device="cuda")
    S = api.partition(ctx, grid, cell_y)

    def l1_of(D, beta):
        f = api.evaluate(ctx, grid, D, beta, xq)
        return float((w_d * (f.double() - ycell).abs()).sum().item()) / area

    out = {"uniform_lattice": []}
    for g in (6, 12, 24, 44):
        D = api.init_lattice(ctx, grid, [g] * grid.dim, g ** grid.dim, wl.sigma_factor)
        o = api.EnetOpts(wl.lambda1, wl.lambda2, prec)
        api.fit(ctx, S, D, o)                  # untimed: workspace sized
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        beta, st = api.fit(ctx, S, D, o)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out["uniform_lattice"].append({"g": g, "centers": g ** grid.dim, "fits_per_s": D.n_sub / dt,
                                       "field_l1_log10": l1_of(D, beta),
                                       "status_ok": bool(np.all(api.stats_to_numpy(st)["status"] == 0))})
    progress("uniform lattices done")
    D = api.init_lattice(ctx, grid, wl.g, m_cap, wl.sigma_factor)
    ro = api.RefineOpts(k_top=wl.k_top, max_rounds=wl.max_rounds, eps_tol=eps, eta=wl.eta, space=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    beta, lvl, rounds, rs, st = api.refine(ctx, S, D, api.EnetOpts(wl.lambda1, wl.lambda2, prec), ro)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["indicator_on_k"] = {"fits": int(rounds.sum().item()), "fits_per_s": int(rounds.sum().item()) / dt,
                             "centers_final_mean": float(D.m.double().mean().item()),
                             "field_l1_log10": l1_of(D, beta)}
    progress("indicator on K done")
    return out


def blend_pairs(grid, m_sub, xq, blend):
    """Query-center pairs of the continuous reconstruction: per query, each
    subdomain with non-zero weight contributes its dictionary size."""
    d = grid.dim
    ax = []
    for a in range(d):
        hcell = (grid.hi[a] - grid.lo[a]) / grid.n_cells[a]
        ax.append(np.array([grid.lo[a] + float(b) * hcell for b in grid.breaks[a]]))
    ns = [len(b) - 1 for b in ax]
    k, nb = [], []
    for a in range(d):
        b, t = ax[a], xq[:, a]
        ka = np.clip(np.searchsorted(b, t, side="right") - 1, 0, ns[a] - 1)
        h = np.zeros(ns[a] + 1)
        for i in range(1, ns[a]):
            h[i] = blend * min(b[i] - b[i - 1], b[i + 1] - b[i])
        right = (ka + 1 < ns[a]) & (t > b[np.minimum(ka + 1, ns[a])] - h[np.minimum(ka + 1, ns[a])])
        left = (ka > 0) & ~right & (t < b[ka] + h[ka])
        k.append(ka)
        nb.append(np.where(right, 1, np.where(left, -1, 0)))
    stride = np.cumprod([1] + ns[:-1])
    pairs = 0.0
    for c in range(1 << d):
        ok = np.ones(len(xq), bool)
        sub = np.zeros(len(xq), np.int64)
        for a in range(d):
            if (c >> a) & 1:
                ok &= nb[a] != 0
                sub += (k[a] + nb[a]) * stride[a]
            else:
                sub += k[a] * stride[a]
        pairs += float(m_sub[sub[ok]].sum())
    return pairs


def continuity(ctx, api, grid, D, beta, xq, w_d, ycell, area, blend, reps=3):
    """Interface treatment on the fitted field: the continuous reconstruction
    timed beside the owner one (HIP events on the library's stream), both
    fields' L1 errors, and the jumps of each across the interfaces."""
    import torch
    Q = int(xq.shape[0])
    ctx.timing(True)
    res = {}
    for name in ("owner", "blend"):
        run = (lambda: api.evaluate(ctx, grid, D, beta, xq)) if name == "owner" else \
            (lambda: api.evaluate_blend(ctx, grid, D, beta, xq, blend))
        out = run()
        torch.cuda.synchronize()
        ctx.timing_read(reset=True)
        for _ in range(reps):
            out = run()
        tk = ctx.timing_read(reset=True)
        ms = (tk["eval_bin"][0] + tk["eval" if name == "owner" else "blend"][0]) / reps
        l1 = float((w_d * (out.double() - ycell).abs()).sum().item()) / area
        res[name] = {"ms": ms, "query_evals_per_s": Q / (ms / 1e3), "field_l1_log10": l1,
                     "kernel_ms": (tk["eval" if name == "owner" else "blend"][0]) / reps}
    ctx.timing(False)
    # jumps: the owner field's interface jump at 64 midpoints per face, and
    # both fields' one-sided differences across the same points
    n = 64 if grid.dim == 2 else 8
    J = api.interface_jump(ctx, grid, D, beta, n).cpu().numpy()
    ax = api.axis_coords(grid)
    pts, nrm = [], []
    ns = [len(b) - 1 for b in ax]
    for a in range(grid.dim):
        for i in range(1, ns[a]):
            others = [b for b in range(grid.dim) if b != a]
            grids1 = [np.linspace(ax[b][0], ax[b][-1], 4 * n * ns[b] + 1)[1:-1] for b in others]
            mesh = np.meshgrid(*grids1, indexing="ij")
            P = np.zeros((mesh[0].size, grid.dim))
            for j, b in enumerate(others):
                P[:, b] = mesh[j].ravel()
            P[:, a] = ax[a][i]
            pts.append(P)
            nrm.append(np.full(len(P), a))
    P, A = np.concatenate(pts), np.concatenate(nrm)
    eps = 1e-7 * float(np.min(grid.cell_size))
    lo, hi = P.copy(), P.copy()
    lo[np.arange(len(P)), A] -= eps
    hi[np.arange(len(P)), A] += eps
    X = torch.as_tensor(np.concatenate([lo, hi]), device=xq.device)
    vo = api.evaluate(ctx, grid, D, beta, X).cpu().numpy()
    vb = api.evaluate_blend(ctx, grid, D, beta, X, blend).cpu().numpy()
    m = len(P)
    pairs = blend_pairs(grid, D.m.cpu().numpy().astype(np.float64), xq.cpu().numpy().astype(np.float64),
                        blend)
    peak_pairs = SLOTS_F32 / 11.0
    ach = pairs / (res["blend"]["kernel_ms"] / 1e3)
    return {
        "blend": blend, "queries": Q,
        "owner": res["owner"], "continuous": res["blend"],
        "interface_jump_owner": {"faces": int(len(J)), "samples_per_face": n ** (grid.dim - 1),
                                 "max": float(J[:, 0].max()), "mean": float(J[:, 1].mean())},
        "one_sided_difference": {"points": m, "eps": eps,
                                 "owner_max": float(np.abs(vo[:m] - vo[m:]).max()),
                                 "continuous_max": float(np.abs(vb[:m] - vb[m:]).max())},
        "roofline": {"bound": "alu", "achieved": ach / 1e12, "peak": peak_pairs / 1e12,
                     "unit": "Tpair/s", "frac": ach / peak_pairs,
                     "kernel": "k_eval_chunks<float, true>", "pairs_per_launch": pairs},
    }


def progress(msg):
    """One line per finished phase on stderr (the JSON result goes to stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs the hot path on one GPU; --gpus {args.gpus} is not "
              "supported (see the sharding notes in DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    progress("importing torch")
    import torch
    progress("torch imported")
    if args.copy_calibration:
        n = 1 << 28
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": 4 * n, "copy_bytes_written_per_launch": 4 * n,
                          "launches": 3}))
        return
    from paper_2605_16564_amd import api, synth

    wl = synth.workload(args.workload)
    prec = args.precision or wl.precision
    grid = wl.grids[0]
    ctx = api.Context(0)
    dev = torch.device("cuda", 0)
    cell_y = torch.as_tensor(grid.y, dtype=torch.float64, device=dev)
    per = 2 ** grid.dim - 1
    m_cap = wl.m0 + wl.max_rounds * wl.k_top * per
    pts, wts, cell_of = synth.metric_points(grid, 4 if grid.dim < 3 else 2)
    xq = torch.as_tensor(pts, dtype=torch.float32, device=dev)
    w_d = torch.as_tensor(wts, dtype=torch.float64, device=dev)
    ycell = cell_y[torch.as_tensor(cell_of, device=dev)]
    Q = xq.shape[0]
    eps = wl.eps_tol_rel * float(np.prod(grid.cell_size))
    use_learned = not args.no_learned and grid.dim == 2
    params, learned_rec = None, None
    if use_learned:
        from paper_2605_16564_amd import learned
        params, learned_rec = train_learned(ctx, api, wl, prec, args.train_mosaics)

    def step(batched=True, cold=False, hinted=use_learned, precision=prec, basis="shepard"):
        S = api.partition(ctx, grid, cell_y)
        D = api.init_lattice(ctx, grid, wl.g, m_cap, wl.sigma_factor, basis=basis)
        hint = learned.hint(ctx, params, grid, D, precision="bf16") if hinted else None
        o = api.EnetOpts(wl.lambda1, wl.lambda2, precision, cd_sweeps=args.cd_sweeps, batched=batched,
                         support_hint=hint)
        ro = api.RefineOpts(k_top=wl.k_top, max_rounds=wl.max_rounds, eps_tol=eps, eta=wl.eta,
                            cold_rounds=cold)
        beta, lvl, rounds, rs, stats = api.refine(ctx, S, D, o, ro)
        out = api.evaluate(ctx, grid, D, beta, xq)
        return S, D, beta, rounds, rs, stats, out

    progress("start" if not use_learned else "learned warm start trained")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.timing(True)
    ctx.timing_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tk = ctx.timing_read(reset=True)
    ctx.timing(False)
    S, D, beta, rounds, rs, stats, out = res
    elapsed = t1 - t0
    ms_step = 1e3 * elapsed / args.steps
    rounds_h = rounds.cpu().numpy()
    rs_h = rs.cpu().numpy()
    st = api.stats_to_numpy(stats)
    fits_step = int(rounds_h.sum())
    value = fits_step * args.steps / elapsed
    # field error of the GPU reconstruction (log10 units), metric quadrature
    area = float(np.prod([grid.hi[a] - grid.lo[a] for a in range(grid.dim)]))
    l1 = float((w_d * (out.double() - ycell).abs()).sum().item()) / area

    # algorithmic work of the timed steps (per step, from the per-round counts)
    n_of = np.diff(S.off_host)
    solve_bytes = float(rs_h[..., 5].sum())
    gram_flops = 0.0
    pairs_design = 0.0
    pairs_ind = 0.0
    for s in range(D.n_sub):
        for r in range(int(rounds_h[s])):
            M = float(rs_h[s, r, 0])
            gram_flops += float(n_of[s]) * (M + 1.0) * (M + 2.0)   # symmetric (M+1)^2 product
            pairs_design += 2.0 * n_of[s] * M                      # two exp passes
            pairs_ind += (2 ** grid.dim) * n_of[s] * M
    m_final = D.m.cpu().numpy().astype(np.float64)
    # queries are the metric points (the same count in every cell), so each
    # subdomain receives its owned cells' share of them
    owned = np.ones(D.n_sub)
    ns = list(grid.n_sub[: grid.dim]) + [1] * (3 - grid.dim)
    s_id = 0
    for k2 in range(ns[2]):
        for k1 in range(ns[1]):
            for k0 in range(ns[0]):
                kk = (k0, k1, k2)
                owned[s_id] = np.prod([grid.breaks[a][kk[a] + 1] - grid.breaks[a][kk[a]]
                                       for a in range(grid.dim)])
                s_id += 1
    eval_pairs = float(np.sum(owned / owned.sum() * Q * m_final))
    per_kernel = {k: {"ms_per_step": v[0] / args.steps, "launches_per_step": v[1] / args.steps}
                  for k, v in tk.items() if v[1] > 0}
    dominant = max(per_kernel, key=lambda k: per_kernel[k]["ms_per_step"])

    def roofline_for(kind):
        ms = per_kernel[kind]["ms_per_step"]
        launches = per_kernel[kind]["launches_per_step"]
        avg_s = ms / 1e3 / launches
        if kind == "gram":
            per_launch = gram_flops / launches
            ach = per_launch / avg_s / 1e12
            peak = PEAK_MFMA[prec]
            return {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                    "frac": ach / peak, "traffic": None, "kernel": "k_gram_" + prec}
        if kind == "eval":
            # FP32 pair = 7 VALU slots + one exp (4 slots)
            peak_pairs = SLOTS_F32 / 11.0
            per_launch = eval_pairs / launches
            ach = per_launch / avg_s
            return {"bound": "alu", "achieved": ach / 1e12, "peak": peak_pairs / 1e12,
                    "unit": "Tpair/s", "frac": ach / peak_pairs, "traffic": None,
                    "kernel": "k_eval_chunks<float>"}
        if kind == "solve":
            # the active-set iteration streams the Gram rows and the inverse of
            # the active block; algorithmic bytes counted by the kernel itself
            per_launch = solve_bytes / launches
            ach = per_launch / avg_s / 1e9
            team = int(st["team"].max()) > 1   # the instance with workgroup teams ran
            kname = "k_solve<" + ("double" if prec == "f64" else "float") + (", true>" if team else ", false>")
            tr = measured_traffic(kname, args.workload)
            return {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": ach / PEAK_HBM_GBS,
                    "traffic": None if tr is None else tr / 1e9,
                    "traffic_unit": "GB per launch",
                    "algorithmic": per_launch / 1e9, "kernel": kname}
        if kind == "indicator":
            # FP64 pair: software exp (about 20 FP64 slots) + 12 others
            peak_pairs = SLOTS_F64 / 32.0
            per_launch = pairs_ind / launches
            ach = per_launch / avg_s
            return {"bound": "alu", "achieved": ach / 1e12, "peak": peak_pairs / 1e12,
                    "unit": "Tpair/s", "frac": ach / peak_pairs, "traffic": None,
                    "kernel": "k_indicator"}
        if kind == "assemble":
            peak_pairs = SLOTS_F64 / 32.0 if prec == "f64" else SLOTS_F32 / 11.0
            per_launch = pairs_design / launches
            ach = per_launch / avg_s
            return {"bound": "alu", "achieved": ach / 1e12, "peak": peak_pairs / 1e12,
                    "unit": "Tpair/s", "frac": ach / peak_pairs, "traffic": None,
                    "kernel": "k_assemble"}
        return None

    roof = roofline_for(dominant) or roofline_for("gram")
    eval_ms = per_kernel.get("eval", {}).get("ms_per_step", float("nan")) + \
        per_kernel.get("eval_bin", {}).get("ms_per_step", 0.0)
    rec = {
        "metric": "subdomain fits/s",
        "value": value,
        "unit": "fits/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {"workload": args.workload, "n_subdomains": int(D.n_sub),
                   "fits_per_step": fits_step, "initial_centers": int(wl.m0),
                   "max_rounds": wl.max_rounds, "k_top": wl.k_top, "queries_per_step": int(Q),
                   "parallelism": "single GPU"},
        "query_evals_per_s": float(Q) / (eval_ms / 1e3) if eval_ms == eval_ms else None,
        "field_l1_log10": l1,
        "kkt_max": float(st["kkt"].max()),
        "fit_status_ok": bool(np.all(st["status"] == 0)),
        "solve_team": int(st["team"].max()),   # workgroups per subdomain in the solve
        "centers_final_mean": float(m_final.mean()),
        "kernels": per_kernel,
        "dominant_kernel": dominant,
        "roofline": roof,
    }
    rec["config"]["learned_warm_start"] = bool(use_learned)
    progress(f"timed steps done: {value:.1f} fits/s")
    if not args.no_select:
        rec["lambda_selection"] = lambda_selection(ctx, api, grid, wl, prec, m_cap, eps, xq, w_d,
                                                   ycell, area, args.select_alphas,
                                                   args.select_folds, args.select_ratio)
    progress("lambda selection done")
    if not args.no_configs:
        rec["other_configs"] = other_configs(ctx, api, synth, progress)
    if not args.no_darcy:
        rec["darcy"] = darcy(ctx, api, grid, D, beta, args.blend)
    progress("Darcy consumer done")
    if not args.no_continuity:
        rec["continuity"] = continuity(ctx, api, grid, D, beta, xq, w_d, ycell, area, args.blend)
    if use_learned:
        learned_rec["gain_first_fit"] = learned_gain(ctx, api, grid, wl, prec, params)
        rec["learned"] = learned_rec
    progress("continuity done")
    if not args.no_ablations:
        # each pattern switched off alone (one untimed and one timed step; the
        # unbatched run is one timed step): fits/s and the ratio it costs
        abl = {}
        variants = [("no_learned", dict(hinted=False), 1), ("fp64", dict(precision="f64"), 1),
                    ("unbatched", dict(batched=False), 0),
                    ("plain_basis", dict(basis="plain", hinted=False), 1)]
        for name, kw, warm in variants:
            if name == "no_learned" and not use_learned:
                continue
            for _ in range(warm):
                step(**kw)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            ra = step(**kw)
            torch.cuda.synchronize()
            va = int(ra[3].sum().item()) / (time.perf_counter() - ta)
            l1a = float((w_d * (ra[6].double() - ycell).abs()).sum().item()) / area
            abl[name] = {"value": va, "unit": "fits/s", "speedup_of_pattern": value / va,
                         "field_l1_log10": l1a}
        rec["ablations"] = abl
    progress("ablations done")
    if not args.no_ablations and not args.no_paper_ablations and grid.dim == 2:
        rec["paper_ablations"] = paper_ablations(ctx, api, grid, wl, prec, m_cap, eps, xq, w_d, ycell,
                                                 area, progress)
    if not args.no_comparator:
        # plain GPU fit: one launch per subdomain and kernel, every refit from
        # zero, no hint; same path otherwise. The per-subdomain launches are
        # serial, so the subdomains are run in two halves (the same work) with
        # a progress line between them
        torch.cuda.synchronize()
        tc0 = time.perf_counter()
        S = api.partition(ctx, grid, cell_y)
        D = api.init_lattice(ctx, grid, wl.g, m_cap, wl.sigma_factor)
        o = api.EnetOpts(wl.lambda1, wl.lambda2, prec, cd_sweeps=args.cd_sweeps, batched=False)
        ro = api.RefineOpts(k_top=wl.k_top, max_rounds=wl.max_rounds, eps_tol=eps, eta=wl.eta,
                            cold_rounds=True)
        half = D.n_sub // 2
        parts = []
        for lo, hi in ((0, half), (half, D.n_sub)):
            Sh, Dh = sub_problem(api, S, D, lo, hi)
            bh, _, rh, _, _ = api.refine(ctx, Sh, Dh, o, ro)
            torch.cuda.synchronize()
            parts.append((Dh, bh, rh))
            progress(f"comparator subdomains {lo}..{hi - 1} done")
        Dc = api.concat_dicts([p_[0] for p_ in parts])
        bc = torch.cat([p_[1] for p_ in parts])
        oc = api.evaluate(ctx, grid, Dc, bc, xq)
        torch.cuda.synchronize()
        tc = time.perf_counter() - tc0
        fits_c = int(sum(int(p_[2].sum().item()) for p_ in parts))
        l1c = float((w_d * (oc.double() - ycell).abs()).sum().item()) / area
        rec["comparator"] = {"kind": "plain GPU fit (per-subdomain launches, cold refits, no hint)",
                             "value": fits_c / tc, "unit": "fits/s", "field_l1_log10": l1c,
                             "speedup": value / (fits_c / tc)}
    progress("comparator done")
    if not args.no_cpu_baseline:
        base, sample = cpu_baseline(grid, wl, args.cpu_sample_subdomains,
                                    min(args.cpu_sample_rounds, wl.max_rounds))
        rec["cpu_baseline"] = base
        rec["oracle_check"] = oracle_check(ctx, api, grid, wl, prec,
                                           api.EnetOpts(wl.lambda1, wl.lambda2, prec), sample)
    print(json.dumps(rec))
    ctx.close()


if __name__ == "__main__":
    main()
