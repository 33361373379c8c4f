"""Timed runs of the FP64 CPU oracle on sampled subdomains of a workload.

TEST INFRASTRUCTURE ONLY: used by the CPU-baseline leg of the benchmark. Each
sampled subdomain runs Alg. 1 (every fit, indicator, marking and enrichment
round) in a worker process of its own with one OpenMP thread, so that the
per-subdomain wall times are one-thread times and the pool's wall time is the
all-core time of the sample. Workers are spawned (never forked) and load only
the oracle and the seeded input generator: they never touch a GPU.
"""
from __future__ import annotations

import os
import platform
import sys
import time
from pathlib import Path


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


_ROOT = str(Path(__file__).resolve().parents[1])


def _init_worker():
    os.environ["OMP_NUM_THREADS"] = "1"
    if _ROOT not in sys.path:
        sys.path.insert(0, _ROOT)


def _refine_one(args):
    """Alg. 1 on one subdomain s of a named workload; returns the timing and
    the oracle's result for that subdomain."""
    name, s = args
    import numpy as np
    from oracle import oracle as O
    from paper_2605_16564_amd import synth
    wl = synth.workload(name)
    g = wl.grids[0]
    S = O.partition(g)
    n_i = np.diff(S["off"])
    per = 2 ** g.dim - 1
    ktop = wl.k_top if wl.k_top else int(np.floor(wl.k_top_frac * n_i[s]))
    k_max = wl.k_top if wl.k_top else int(np.floor(wl.k_top_frac * n_i.max()))
    m_cap = wl.m0 + wl.max_rounds * k_max * per
    D = O.init_dictionary(g, wl.g, m_cap, wl.sigma_factor)
    j0, j1 = S["off"][s], S["off"][s + 1]
    sub = dict(off=np.array([0, j1 - j0], np.int64), x=S["x"][j0:j1], y=S["y"][j0:j1], h=S["h"][j0:j1])
    D1 = O.Dictionary(1, m_cap, g.dim)
    D1.m[:] = D.m[s]
    D1.c[:] = D.c[s * m_cap * g.dim:(s + 1) * m_cap * g.dim]
    D1.sigma[:] = D.sigma[s * m_cap:(s + 1) * m_cap]
    D1.level[:] = D.level[s * m_cap:(s + 1) * m_cap]
    eps = wl.eps_tol_rel * float(np.prod(g.cell_size))
    t0 = time.perf_counter()
    Do, bo, lvl, info = O.refine_batch(sub, D1, wl.lambda1, wl.lambda2, k_top=ktop,
                                       max_rounds=wl.max_rounds, m_max=1 << 30, eps_tol=eps)
    dt = time.perf_counter() - t0
    M = int(Do.m[0])
    return dict(sub=s, seconds=dt, fits=int(info["rounds"][0]), status=int(info["status"][0]),
                m=M, c=Do.c[:M * g.dim].copy(), sigma=Do.sigma[:M].copy(),
                level=Do.level[:M].copy(), beta=bo[:M].copy(), elem_level=lvl.copy(),
                round_stats=info["round_stats"][0].copy())


def pool(workers: int):
    """Spawn the worker processes now (before the caller touches a GPU; the
    workers never do): a multiprocessing pool of `workers` fresh
    interpreters, one OpenMP thread each."""
    import multiprocessing as mp
    return mp.get_context("spawn").Pool(processes=workers, initializer=_init_worker)


def start(pl, name: str, subs, workers: int):
    """Queue the sample on the pool; returns a handle for finish()."""
    t0 = time.perf_counter()
    jobs = [pl.apply_async(_refine_one, ((name, int(s)),)) for s in subs]
    return dict(pool=pl, jobs=jobs, t0=t0, workers=workers, name=name)


def finish(h):
    """Wait for the sample: (record, per-subdomain oracle results)."""
    res = [j.get() for j in h["jobs"]]
    wall = time.perf_counter() - h["t0"]
    h["pool"].close()
    h["pool"].join()
    fits = sum(r["fits"] for r in res)
    busy = sum(r["seconds"] for r in res)
    rec = {"value": fits / wall, "unit": "subdomain fits/s", "cores": min(h["workers"], len(res)),
           "kind": "oracle",
           "one_thread_value": fits / busy,
           "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
           "sample": f"Alg. 1 with every round (fit, indicator, marking, enrichment) on {len(res)} "
                     f"sampled subdomains of {h['name']} ({fits} fits, FP64), one worker process "
                     f"and one thread per subdomain, {min(h['workers'], len(res))} at a time: "
                     f"value = fits / pool wall time ({wall:.1f} s), one_thread_value = fits / "
                     f"summed per-subdomain time ({busy:.1f} s)",
           "wall_s": wall, "busy_s": busy}
    return rec, res
