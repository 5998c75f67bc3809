"""Serving driver: a Poisson stream of simulation requests of mixed N and
grid size fed to the continuous-batching server of the C ABI
(nplbm_server_*), reporting p50/p99 time-to-completion and aggregate MLUPS.

Request layouts come from the seeded ``workloads`` generators (N=3 static
droplet, N=4 droplet collision, N=5 bands and droplets, scaled to the
request's side).  All inputs are generated before the clock starts.
"""
from __future__ import annotations

import time
from typing import Callable, Optional

import numpy as np

from . import nplbm as P


def _prepare(reqs, steps_scale):
    import workloads as W
    jobs = []
    for r in reqs:
        w = W.request_workload(r, accept=P.accepts)
        steps = max(1, int(round(r.steps * steps_scale)))
        jobs.append((r, w, steps))
    return jobs


def _submit(srv, w, steps):
    return srv.submit(w.c, w.u, nsteps=steps, precision=32, **w.params())


def run_stream(nreq: int = 96, steps_scale: float = 0.1, load: float = 0.7,
               budget: int = 8 << 30, quantum: int = 50, max_slots: int = 256,
               seed: Optional[int] = None, log: Callable = print) -> dict:
    import torch
    import workloads as W

    seed = W.BASE_SEED + 5 if seed is None else seed
    reqs = W.request_stream(n=nreq, rate=1.0, seed=seed)
    t0 = time.perf_counter()
    jobs = _prepare(reqs, steps_scale)
    log(f"[serving] prepared {len(jobs)} requests in {time.perf_counter() - t0:.1f} s")
    work = np.array([w.nx * w.ny * s for _, w, s in jobs], dtype=np.float64)

    # warm-up: the first 16 requests at once, to measure batched throughput
    srv = P.Server(hbm_budget=budget, max_slots=max_slots, quantum=quantum)
    tk = [_submit(srv, w, s) for _, w, s in jobs[:16]]
    t0 = time.perf_counter()
    pending = set(tk)
    while pending:
        srv.pump()
        for t in list(pending):
            if srv.poll(t) >= 2:
                srv.result(t)
                pending.discard(t)
    warm_mlups = float(work[:16].sum() / (time.perf_counter() - t0) / 1e6)
    srv.close()

    # arrival rate so that the offered work is `load` of the measured throughput
    rate = load * warm_mlups * 1e6 / float(work.mean())
    arrivals = np.array([r.arrival for r in reqs]) / rate
    log(f"[serving] warm-up {warm_mlups:.0f} MLUPS -> arrival rate {rate:.2f}/s")

    srv = P.Server(hbm_budget=budget, max_slots=max_slots, quantum=quantum)
    torch.cuda.synchronize()
    lat = np.zeros(len(jobs))
    submit_lag = np.zeros(len(jobs))
    tick = {}
    nxt = 0
    done = 0
    max_res = 0
    start = time.perf_counter()
    while done < len(jobs):
        now = time.perf_counter() - start
        while nxt < len(jobs) and arrivals[nxt] <= now:
            _, w, s = jobs[nxt]
            tick[_submit(srv, w, s)] = nxt
            submit_lag[nxt] = (time.perf_counter() - start) - arrivals[nxt]
            nxt += 1
        if not tick and nxt < len(jobs):
            time.sleep(max(0.0, arrivals[nxt] - (time.perf_counter() - start)))
            continue
        active = srv.pump()
        max_res = max(max_res, active)
        for t in list(tick):
            if srv.poll(t) >= 2:
                i = tick.pop(t)
                _, _, _, adm, fin = srv.result(t)
                lat[i] = submit_lag[i] + fin
                done += 1
    makespan = time.perf_counter() - start
    nu, busy, completed = srv.stats()
    srv.close()
    res = {"requests": len(jobs), "p50_s": float(np.percentile(lat, 50)),
           "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()),
           "aggregate_mlups": float(work.sum() / makespan / 1e6),
           "makespan_s": makespan, "arrival_rate_per_s": rate, "offered_load": load,
           "warmup_batched_mlups": warm_mlups, "hbm_budget_bytes": budget, "quantum": quantum,
           "max_resident": int(max_res), "steps_scale": steps_scale,
           "precision": "fp32"}
    log(f"[serving] p50 {res['p50_s']:.3f} s p99 {res['p99_s']:.3f} s "
        f"aggregate {res['aggregate_mlups']:.0f} MLUPS")
    return res
