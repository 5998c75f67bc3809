"""Serving: continuous batching of mixed-N, mixed-size domains gives the
same result for every request as running it alone (bitwise, FP32), with
requests admitted while others are resident and finishing mid-quantum, and
every served FP64 request matches the FP64 oracle (1e-10 max-abs)."""
import numpy as np
import pytest

import workloads as W
from gpu_util import maxabs, oracle_run

pytestmark = pytest.mark.gpu


def _alone(w, steps):
    import paper_1904_12553_amd as P
    d = P.Domain(precision=32, **w.params())
    d.set_fields(w.c, w.u)
    d.step(steps)
    return d.macro()


def test_alone_equals_mix():
    import paper_1904_12553_amd as P
    reqs = [W.Request(i, 0.0, N, side, steps, W.BASE_SEED * 10 + i)
            for i, (N, side, steps) in enumerate([(3, 64, 37), (4, 96, 120), (5, 128, 75),
                                                   (3, 80, 200), (5, 64, 13), (4, 64, 90)])]
    ws = [W.request_workload(r, accept=P.accepts) for r in reqs]
    srv = P.Server(hbm_budget=1 << 30, max_slots=4, quantum=16)
    tickets = []
    # first three now, the rest after two quanta (admitted into a running mix)
    for r, w in list(zip(reqs, ws))[:3]:
        tickets.append(srv.submit(w.c, w.u, nsteps=r.steps, precision=32, **w.params()))
    srv.pump()
    srv.pump()
    for r, w in list(zip(reqs, ws))[3:]:
        tickets.append(srv.submit(w.c, w.u, nsteps=r.steps, precision=32, **w.params()))
    results = {}
    for _ in range(1000):
        srv.pump()
        for t in tickets:
            if t not in results and srv.poll(t) == 2:
                results[t] = srv.result(t)
        if len(results) == len(tickets):
            break
    assert len(results) == len(tickets)
    for t, r, w in zip(tickets, reqs, ws):
        c, u, p, adm, fin = results[t]
        ca, ua, pa = _alone(w, r.steps)
        assert np.array_equal(c, ca) and np.array_equal(u, ua) and np.array_equal(p, pa), r
        assert fin >= adm >= 0.0
    st = srv.stats()
    assert st["completed"] == len(reqs)
    assert st["node_updates"] == pytest.approx(sum(w.nx * w.ny * r.steps for r, w in zip(reqs, ws)))
    # the library's latency percentiles and throughput
    lat = sorted(results[t][4] for t in tickets)
    assert 0.0 < st["p50_s"] <= st["p99_s"] <= lat[-1] + 1e-9
    assert st["p50_s"] == pytest.approx(float(np.percentile(lat, 50)), rel=1e-9)
    assert st["p99_s"] == pytest.approx(float(np.percentile(lat, 99)), rel=1e-9)
    assert st["mlups"] > 0.0


def test_budget_admission_and_too_big():
    import paper_1904_12553_amd as P
    w = W.static_droplet(64, 64, R=16, precision=32)
    fp = P.footprint(precision=32, **w.params())
    srv = P.Server(hbm_budget=int(fp * 1.5), max_slots=8, quantum=10)
    t1 = srv.submit(w.c, None, nsteps=30, precision=32, **w.params())
    t2 = srv.submit(w.c, None, nsteps=30, precision=32, **w.params())
    srv.pump()
    assert srv.poll(t1) == 1 and srv.poll(t2) == 0   # only one fits the budget
    # asking too early is an error that keeps the ticket
    with pytest.raises(P.NplbmError) as e:
        srv.result(t2)
    assert e.value.code == -6 and srv.poll(t2) == 0
    big = W.static_droplet(128, 128, R=30, precision=32)
    with pytest.raises(P.NplbmError) as e:
        srv.submit(big.c, None, nsteps=10, precision=32, **big.params())
    assert e.value.code == -5
    for _ in range(20):
        srv.pump()
    assert srv.poll(t1) == 2 and srv.poll(t2) == 2
    for t in (t1, t2):
        c, _, _, _, _ = srv.result(t)
        assert np.all(np.isfinite(c))
    with pytest.raises(P.NplbmError) as e:           # collected once only
        srv.result(t1)
    assert e.value.code == -7


def test_served_fp64_requests_match_the_oracle():
    """FP64 requests of the three schemes, periodic and with walls, served in
    a mix with FP32 requests: two are admitted into the running mix, most
    finish in the middle of a quantum; each one's c, u and p match the FP64
    oracle run of the same request within 1e-10 max-abs."""
    import paper_1904_12553_amd as P
    from oracle.accept import oracle_accepts
    mk = lambda N, nx, ny, seed, wall: W.random_smooth(N, nx, ny, seed=seed, wall_y=wall,
                                                       accept=oracle_accepts)
    first = [(mk(3, 48, 40, 901, False), {}, 64, 70),
             (mk(4, 40, 36, 902, True), {"grad_scheme": 1}, 64, 53),
             (mk(2, 36, 30, 903, True), {"force_form": 1}, 64, 45),
             (mk(5, 64, 64, 904, False), {}, 32, 100)]
    later = [(mk(5, 44, 40, 905, True), {}, 64, 37),
             (mk(3, 50, 30, 906, False), {"force_form": 1}, 64, 21),
             (mk(4, 33, 20, 907, False), {"grad_scheme": 1}, 32, 29)]
    print("case served FP64 vs oracle: " + ", ".join(
        f"N={w.N} {w.nx}x{w.ny} {o} fp{p} {s}" for w, o, p, s in first + later), flush=True)
    srv = P.Server(hbm_budget=1 << 31, max_slots=8, quantum=16)
    tickets = {}
    for job in first:
        w, over, prec, steps = job
        tickets[srv.submit(w.c, w.u, nsteps=steps, precision=prec,
                           **dict(w.params(), **over))] = job
    srv.pump()
    srv.pump()                      # 32 steps into the first requests
    for job in later:
        w, over, prec, steps = job
        tickets[srv.submit(w.c, w.u, nsteps=steps, precision=prec,
                           **dict(w.params(), **over))] = job
    results = {}
    for _ in range(200):
        srv.pump()
        for t in tickets:
            if t not in results and srv.poll(t) == 2:
                results[t] = srv.result(t)
        if len(results) == len(tickets):
            break
    srv.close()
    assert len(results) == len(tickets)
    checked = 0
    for t, (w, over, prec, steps) in tickets.items():
        if prec != 64:
            continue
        c, u, p, _, _ = results[t]
        o = oracle_run(w, steps, **over)
        oc, ou, op = o.macro()
        err = max(maxabs(c, oc), maxabs(u, ou), maxabs(p, op))
        assert err < 1e-10, (w.N, w.nx, w.ny, over, steps, err)
        checked += 1
    assert checked == 5


def test_server_in_a_fresh_process_that_loads_the_library_first():
    # the library is loaded (by the tension check) before anything else
    # touches the GPU; the server must still find the device
    import os
    import subprocess
    import sys
    code = ("import paper_1904_12553_amd as P, workloads as W; "
            "w = W.static_droplet(64, 64, R=16); assert P.accepts(w.sigma, w.rho); "
            "s = P.Server(hbm_budget=1 << 30, max_slots=2, quantum=8); "
            "t = s.submit(w.c, w.u, nsteps=20, precision=32, **w.params()); "
            "[s.pump() for _ in range(5)]; assert s.poll(t) == 2; s.result(t); s.close(); "
            "print('server ok')")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    print("case fresh-process server", flush=True)
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                       timeout=200, env=dict(os.environ, PYTHONPATH=root))
    assert r.returncode == 0 and "server ok" in r.stdout, r.stdout + r.stderr


@pytest.mark.parametrize("seed", range(3))
def test_seeded_mixes_alone_equals_mix(seed):
    """Seeded mixes of 8 requests over N = 2..8, the three schemes, both
    precisions, periodic or walls, sides 20..150, 1..120 steps, arriving
    in three waves (into a running mix, so groups appear and vanish between
    quanta): every result bitwise equal to the request run alone."""
    import paper_1904_12553_amd as P
    rng = np.random.default_rng(300 + seed)
    jobs = []
    for i in range(8):
        N = int(rng.integers(2, 9))
        nx, ny = int(rng.integers(20, 151)), int(rng.integers(8, 121))
        wall = bool(rng.integers(0, 2))
        sig = (0.5e-3, 2e-3) if N <= 5 else (0.8e-3, 1.2e-3)
        w = W.random_smooth(N, nx, ny, seed=3000 + 10 * seed + i, wall_y=wall,
                            accept=P.accepts, sigma_range=sig)
        over = [{}, {"grad_scheme": 1}, {"force_form": 1}][int(rng.integers(0, 3))]
        prec = int(rng.choice([32, 64]))
        steps = int(rng.integers(1, 121))
        jobs.append((w, over, prec, steps))
    print(f"case seeded mix {seed}: " + ", ".join(
        f"N={w.N} {w.nx}x{w.ny} {o} fp{p} {s}" for w, o, p, s in jobs), flush=True)
    srv = P.Server(hbm_budget=1 << 31, max_slots=6, quantum=20)
    tickets = {}
    for wave in (jobs[:3], jobs[3:6], jobs[6:]):
        for w, over, prec, steps in wave:
            tickets[srv.submit(w.c, w.u, nsteps=steps, precision=prec,
                               **dict(w.params(), **over))] = (w, over, prec, steps)
        srv.pump()
    results = {}
    for _ in range(2000):
        srv.pump()
        for t in tickets:
            if t not in results and srv.poll(t) == 2:
                results[t] = srv.result(t)
        if len(results) == len(tickets):
            break
    srv.close()
    assert len(results) == len(tickets)
    for t, (w, over, prec, steps) in tickets.items():
        d = P.Domain(precision=prec, **dict(w.params(), **over))
        d.set_fields(w.c, w.u)
        d.step(steps)
        ca, ua, pa = d.macro()
        d.close()
        c, u, p, _, _ = results[t]
        assert np.array_equal(c, ca) and np.array_equal(u, ua) and np.array_equal(p, pa), \
            (w.N, w.nx, w.ny, over, prec, steps)


def test_submit_from_threads_while_pumping():
    """Four threads submit four requests each while the main thread pumps
    and a fifth thread polls every ticket (submit and poll are thread-safe;
    the binding's foreign calls release the GIL): every ticket is distinct,
    the states a ticket shows only move forward (queued, resident, done),
    and every result is bitwise the request alone."""
    import threading

    import paper_1904_12553_amd as P
    rng = np.random.default_rng(77)
    jobs = []
    for i in range(16):
        N = int(rng.integers(2, 6))
        w = W.random_smooth(N, int(rng.integers(20, 90)), int(rng.integers(8, 60)),
                            seed=4000 + i, wall_y=bool(i % 2), accept=P.accepts)
        jobs.append((w, int(rng.integers(5, 60))))
    print("case threaded submit 4 x 4", flush=True)
    srv = P.Server(hbm_budget=1 << 31, max_slots=8, quantum=10)
    tickets = [None] * len(jobs)

    def submitter(k):
        for i in range(k, len(jobs), 4):
            w, steps = jobs[i]
            tickets[i] = srv.submit(w.c, w.u, nsteps=steps, precision=32, **w.params())

    seen, errors = {}, []
    stop = threading.Event()

    def poller():
        while not stop.is_set():
            for t in list(tickets):
                if t is None or seen.get(t, [None])[-1] in (2, "gone"):
                    continue
                try:
                    st = srv.poll(t)
                except P.NplbmError as e:   # result() already took it
                    if e.code != -7:
                        errors.append(e)
                    st = "gone"
                if seen.setdefault(t, [st])[-1] != st:
                    seen[t].append(st)

    threads = [threading.Thread(target=submitter, args=(k,)) for k in range(4)]
    threads.append(threading.Thread(target=poller, daemon=True))
    for t in threads:
        t.start()
    results = {}
    try:
        for _ in range(3000):
            srv.pump()
            for t in tickets:
                if t is not None and t not in results and srv.poll(t) == 2:
                    results[t] = srv.result(t)
            if all(t is not None for t in tickets) and len(results) == len(jobs):
                break
    finally:
        stop.set()
        for t in threads:
            t.join()
    srv.close()
    assert not errors, errors
    assert len(set(tickets)) == len(jobs) and len(results) == len(jobs)
    order = {0: 0, 1: 1, 2: 2, "gone": 3}
    for t, states in seen.items():
        ranks = [order[x] for x in states]
        assert ranks == sorted(ranks) and 3 not in states, (t, states)
    for t, (w, steps) in zip(tickets, jobs):
        ca, ua, pa = _alone(w, steps)
        c, u, p, _, _ = results[t]
        assert np.array_equal(c, ca) and np.array_equal(u, ua) and np.array_equal(p, pa)
