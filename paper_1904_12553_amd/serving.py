"""Serving driver: a Poisson stream of simulation requests of mixed N and
grid size fed to the continuous-batching server of the C ABI
(nplbm_server_*).

A submitter thread calls ``nplbm_submit`` at each request's arrival time
(submission is thread-safe and the binding's foreign calls release the GIL)
while the main thread pumps the server and collects finished requests, so
requests arrive while others are resident on the GPU.  The p50/p99
time-to-completion (submission to completion) and the aggregate MLUPS are
the library's own (``nplbm_server_stats``).

Request layouts come from the seeded ``workloads`` generators (N=3 static
droplet, N=4 droplet collision, N=5 bands and droplets, scaled to the
request's side).  All inputs are generated before the clock starts.
"""
from __future__ import annotations

import threading
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


def _drain(srv, tickets, failed):
    """Collect every finished ticket; returns how many finished."""
    n = 0
    for t in list(tickets):
        if srv.poll(t) >= 2:
            tickets.discard(t)
            n += 1
            try:
                srv.result(t)
            except P.NplbmError:
                failed.append(t)
    return n


def warmup_throughput(jobs, budget, quantum, max_slots, n=16):
    """Batched throughput of the first n requests submitted at once (MLUPS)."""
    srv = P.Server(hbm_budget=budget, max_slots=max_slots, quantum=quantum)
    pending = {_submit(srv, w, s) for _, w, s in jobs[:n]}
    failed = []
    while pending:
        srv.pump()
        _drain(srv, pending, failed)
    st = srv.stats()
    srv.close()
    if failed:
        raise RuntimeError(f"{len(failed)} warm-up requests failed")
    return st["mlups"]


def run_stream(nreq: int = 512, steps_scale: float = 1.0, load: float = 0.7,
               budget: int = 8 << 30, quantum: int = 50, max_slots: int = 256,
               seed: Optional[int] = None, rate: Optional[float] = None,
               jobs=None, log: Callable = print) -> dict:
    """Serve a seeded Poisson stream of ``nreq`` requests.  The arrival rate
    is ``rate`` if given, else ``load`` times the batched throughput of a
    warm-up over the mean work of a request."""
    import torch
    import workloads as W

    seed = W.BASE_SEED + 5 if seed is None else seed
    reqs = W.request_stream(n=nreq, rate=1.0, seed=seed)
    if jobs is None:
        t0 = time.perf_counter()
        jobs = _prepare(reqs, steps_scale)
        log(f"[serving] prepared {len(jobs)} requests in {time.perf_counter() - t0:.1f} s")
    work = np.array([w.nx * w.ny * s for _, w, s in jobs], dtype=np.float64)
    warm = None
    if rate is None:
        warm = warmup_throughput(jobs, budget, quantum, max_slots)
        rate = load * warm * 1e6 / float(work.mean())
        log(f"[serving] warm-up {warm:.0f} MLUPS -> arrival rate {rate:.2f}/s")
    arrivals = np.array([r.arrival for r in reqs]) / rate

    srv = P.Server(hbm_budget=budget, max_slots=max_slots, quantum=quantum)
    torch.cuda.synchronize()
    tickets: set = set()
    lock = threading.Lock()
    lag = np.zeros(len(jobs))
    errors = []
    start = time.perf_counter()

    def submitter():
        try:
            for i, (_, w, s) in enumerate(jobs):
                wait = arrivals[i] - (time.perf_counter() - start)
                if wait > 0:
                    time.sleep(wait)
                lag[i] = (time.perf_counter() - start) - arrivals[i]
                t = _submit(srv, w, s)
                with lock:
                    tickets.add(t)
        except Exception as e:  # surfaced by the main thread
            errors.append(e)

    th = threading.Thread(target=submitter)
    th.start()
    done = 0
    failed = []
    max_res = 0
    while done + len(failed) < len(jobs) and not errors:
        active = srv.pump()
        max_res = max(max_res, active)
        with lock:
            live = set(tickets)
        before = len(live)
        nfin = 0
        for t in list(live):
            if srv.poll(t) >= 2:
                with lock:
                    tickets.discard(t)
                try:
                    srv.result(t)
                    nfin += 1
                except P.NplbmError:
                    failed.append(t)
        done += nfin
        if active == 0 and before == 0:
            time.sleep(0.0005)        # nothing resident or queued: wait for an arrival
    th.join()
    if errors:
        raise errors[0]
    makespan = time.perf_counter() - start
    st = srv.stats()
    srv.close()
    res = {"requests": len(jobs), "completed": int(st["completed"]), "failed": len(failed),
           "p50_s": st["p50_s"], "p99_s": st["p99_s"], "aggregate_mlups": st["mlups"],
           "makespan_s": makespan, "arrival_rate_per_s": rate, "offered_load": load,
           "warmup_batched_mlups": warm, "hbm_budget_bytes": int(budget), "quantum": quantum,
           "max_resident": int(max_res), "steps_scale": steps_scale,
           "submit_lag_p99_s": float(np.percentile(lag, 99)), "precision": "fp32"}
    log(f"[serving] budget {budget / 2**30:.0f} GiB: p50 {res['p50_s']:.3f} s "
        f"p99 {res['p99_s']:.3f} s aggregate {res['aggregate_mlups']:.0f} MLUPS, "
        f"makespan {makespan:.1f} s, up to {max_res} resident")
    return res
