"""Benchmark of the fused N-phase LB step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-serving]

Workload (one "step" = one pass of the whole hot path): the N=5 droplets and
interfaces configuration -- 2048 x 2048 periodic lattice, four stacked bands
of phases 1-4 plus 64 seeded phase-5 droplets (r ~ U[10, 40]), sigma_kl ~
U[0.5e-3, 2e-3] (SPD-checked), rho_k ~ U[1, 3], FP32 state -- advanced by
the fused step kernel (replayed as HIP graphs), with the FP64 conservation
diagnostics (per-phase mass, max |sum c - 1|, non-finite count) every 100
steps and at the end of the timed region, inside it.  Inputs are resident
in HBM before timing starts.

Prints ONE JSON line: MLUPS (node updates per second / 1e6), the roofline
object of the step kernel (algorithmic bytes 20 N s per node update over the
kernel's average duration, measured with HIP events on the stream the kernel
runs on, beside the measured device-copy bandwidth), the FP64 run of the
same workload and its speedup, the FP32-vs-FP64 error on c after a short
window, mass drift, the other phase counts and the D3Q15 workloads, the
serving stream of the workload table (512 Poisson requests, 1000-20000
steps, at an 8 GiB budget and at the whole free device memory: p50/p99
time-to-completion and aggregate MLUPS from the library) and the FP64 CPU
oracle timed on the host (single thread and all cores, over the workload
table's windows).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
DIAG_EVERY = 100


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash():
    """Hash of the step kernel's code (its sources with comments and
    whitespace removed), so that the committed counter record is used only
    for the code it was taken on."""
    h = hashlib.sha256()
    for f in ("step_kernel.hip", "buffer_io.h", "nplbm_internal.h", "lattice.h"):
        with open(os.path.join(ROOT, "paper_1904_12553_amd", "csrc", f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def traffic_from_profiles(nodes):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    or None if the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "step_kernel_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_hash") != kernel_hash() or t.get("nodes") != nodes:
        return None
    return t.get("bytes_per_launch")


def time_steps(d, steps, torch, diag_every=DIAG_EVERY):
    """Run `steps` steps with the FP64 diagnostics every `diag_every` steps
    and after the last one; returns (wall seconds, summed step seconds from
    HIP events on the domain's stream, last diagnostics, diagnostics run)."""
    ev = []
    diag = None
    ndiag = 0
    done = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while done < steps:
        n = min(diag_every - done % diag_every, steps - done)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(d.stream)
        d.step(n)
        b.record(d.stream)
        ev.append((a, b))
        done += n
        if done % diag_every == 0 or done == steps:
            diag = d.diagnostics()
            ndiag += 1
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern = sum(a.elapsed_time(b) for a, b in ev) / 1e3
    return wall, kern, diag, ndiag


def kernel_rate(P, w, prec, steps, torch, **over):
    """Step-kernel time of a workload (HIP events around `steps` steps after
    a warmup): ms per step, MLUPS and the fraction of the HBM roofline with
    the algorithmic bytes per node update -- 20 N s on D2Q9, 2 (16 N + 1) s
    on D3Q15 -- for state word size s."""
    d = P.Domain(precision=prec, **dict(w.params(), **over))
    d.set_fields(w.c, w.u)
    d.step(steps)
    d.sync()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(d.stream)
    d.step(steps)
    b.record(d.stream)
    b.synchronize()
    ms = a.elapsed_time(b) / steps
    nodes = d.n
    s = 8 if prec == 64 else 4
    B = (2 * (16 * w.N + 1) if d.dim == 3 else 20 * w.N) * s
    d.close()
    return {"kernel_ms": round(ms, 5), "MLUPS": round(nodes / ms / 1e3, 1),
            "bytes_per_node_update": B,
            "roofline_frac": round(nodes * B / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def copy_bandwidth(P, torch, mib=1024, reps=20):
    """Read + write bandwidth of the library's plain copy kernel (GB/s)."""
    n = mib << 20
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty(n, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    st = torch.cuda.current_stream()
    for _ in range(3):
        P.device_copy(b, a, n, st)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        P.device_copy(b, a, n, st)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return round(2 * n / ms / 1e6, 1)


# ---------------------------------------------------------------- CPU oracle
# The workload table's windows for timing the oracle (FP64, plain C): the
# static droplet in full, the lens, the droplet collision and the benchmark
# workload over shorter windows.
CPU_WINDOWS = {
    "static_droplet_N3_100x100": ("static", 2000),
    "liquid_lens_N3_400x200": ("lens", 2000),
    "droplet_collision_N4_512x512": ("collision", 500),
    "bands_and_droplets_N5_2048x2048": ("bands", 50),
}


def _cpu_workload(kind):
    import workloads as W
    from oracle.accept import oracle_accepts
    if kind == "static":
        return W.static_droplet()
    if kind == "lens":
        return W.liquid_lens(s12=1e-3, s13=0.8e-3, s23=0.8e-3)
    if kind == "collision":
        return W.droplet_collision(512, accept=oracle_accepts, precision=64)
    return W.bands_and_droplets(2048, accept=oracle_accepts, precision=64)


def cpu_sample(kind, steps):
    """Time `steps` oracle steps of one workload in this process (the thread
    count is OMP_NUM_THREADS); prints one JSON line."""
    from oracle import OracleSim
    w = _cpu_workload(kind)
    o = OracleSim(**w.params())
    o.init(w.c, w.u)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    print(json.dumps({"kind": kind, "steps": steps, "nodes": w.nx * w.ny, "seconds": dt,
                      "MLUPS": w.nx * w.ny * steps / dt / 1e6}), flush=True)


def run_cpu_sample(kind, steps, threads):
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-sample", kind,
                        "--cpu-steps", str(steps)], env=env, capture_output=True, text=True,
                       timeout=600)
    if r.returncode != 0:
        raise RuntimeError(f"CPU sample {kind} failed:\n{r.stderr[-2000:]}")
    return json.loads(r.stdout.strip().splitlines()[-1])


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(single_steps):
    """The oracle on the host: all cores over each window of CPU_WINDOWS, and
    one thread on a few steps of the benchmark workload."""
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    windows = []
    for name, (kind, steps) in CPU_WINDOWS.items():
        r = run_cpu_sample(kind, steps, cores)
        windows.append({"workload": name, "steps": steps, "MLUPS": round(r["MLUPS"], 3),
                        "seconds": round(r["seconds"], 2)})
        log(f"[bench] cpu oracle {name}, {steps} steps, {cores} threads: "
            f"{r['MLUPS']:.2f} MLUPS ({r['seconds']:.1f} s)")
    one = run_cpu_sample("bands", single_steps, 1)
    log(f"[bench] cpu oracle bands, {single_steps} steps, 1 thread: {one['MLUPS']:.3f} MLUPS")
    head = windows[-1]
    return {"value": head["MLUPS"], "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{head['steps']} FP64 steps of the 2048x2048 N=5 workload "
                      f"({head['seconds']} s, {cores} threads)",
            "cpu_model": cpu_model(),
            "single_thread": {"value": round(one["MLUPS"], 4), "unit": "MLUPS", "cores": 1,
                              "sample": f"{single_steps} FP64 steps of the 2048x2048 N=5 "
                                        f"workload ({one['seconds']:.1f} s)"},
            "windows_all_cores": windows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2048)
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--side", type=int, default=2048)
    ap.add_argument("--fp64-steps", type=int, default=512)
    ap.add_argument("--acc-steps", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-single-steps", type=int, default=2)
    ap.add_argument("--cpu-sample", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-steps", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=512)
    ap.add_argument("--serving-steps-scale", type=float, default=1.0)
    ap.add_argument("--serving-budgets", default="8,device",
                    help="comma list of HBM budgets: GiB, or 'device' for the free device memory")
    ap.add_argument("--profile-only", action="store_true",
                    help="only the warmup and timed FP32 steps (for rocprofv3 runs)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the N = 3 / 4 sweep, the Remark 1 and the D3Q15 legs")
    args = ap.parse_args()

    if args.cpu_sample:
        cpu_sample(args.cpu_sample, args.cpu_steps)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the domain and the serving "
                                   "loop live on a single MI355X; multi-GPU slab decomposition "
                                   "is a design note, not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_1904_12553_amd as P
    import workloads as W
    from paper_1904_12553_amd import serving as S

    torch.cuda.set_device(0)
    side = args.side
    log(f"[bench] building workload N=5 {side}x{side}")
    w = W.bands_and_droplets(side, ndrop=64 if side == 2048 else max(4, 64 * side * side // 2048 ** 2),
                             accept=P.accepts)
    nodes = w.nx * w.ny
    B_node = 20 * w.N * 4

    # ---- FP32 timed run ----
    d = P.Domain(precision=32, **w.params())
    d.set_fields(w.c, w.u)
    m0, _, _ = d.diagnostics()
    d.step(args.warmup)
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} done; timing {args.steps} steps")
    wall, kern, diag, ndiag = time_steps(d, args.steps, torch)
    mlups = nodes * args.steps / wall / 1e6
    ms_step = wall / args.steps * 1e3
    k_ms = kern / args.steps * 1e3
    achieved = B_node * nodes / (k_ms * 1e-3) / 1e9
    log(f"[bench] fp32 {mlups:.0f} MLUPS, {ms_step:.4f} ms/step, kernel {k_ms:.4f} ms, "
        f"{achieved:.0f} GB/s, {ndiag} diagnostics in the timed region")
    drift = float(np.max(np.abs(diag[0] - m0) / np.abs(m0)))
    if args.profile_only:
        print(json.dumps({"metric": "MLUPS", "value": round(mlups, 1), "profile_only": True,
                          "kernel_ms": round(k_ms, 5)}))
        return
    d.close()
    del d

    out = {
        "metric": "MLUPS (N=5, FP32, fused step; FP64 diagnostics every 100 steps and at the "
                  "end of the timed region)",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"bands_and_droplets_N5_{side}x{side}_periodic", "N": 5,
                   "nx": side, "ny": side, "precision": "fp32", "droplets": 64,
                   "diag_every": DIAG_EVERY, "diagnostics_in_timed_region": ndiag},
    }
    copy_gbs = copy_bandwidth(P, torch)
    log(f"[bench] device copy {copy_gbs:.0f} GB/s (read + write)")
    traffic = traffic_from_profiles(nodes)
    out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                       "traffic": traffic,
                       "bytes_per_node_update": B_node, "kernel_ms": round(k_ms, 5),
                       "copy_GBps": copy_gbs,
                       "frac_of_copy": round(achieved / copy_gbs, 4)}
    out["mass_drift_rel"] = drift

    # ---- FP64 run of the same workload ----
    d64 = P.Domain(precision=64, **w.params())
    d64.set_fields(w.c, w.u)
    d64.step(args.warmup)
    wall64, kern64, _, _ = time_steps(d64, args.fp64_steps, torch)
    mlups64 = nodes * args.fp64_steps / wall64 / 1e6
    k64 = kern64 / args.fp64_steps * 1e3
    out["fp64"] = {"value": round(mlups64, 1), "unit": "MLUPS",
                   "kernel_ms": round(k64, 5),
                   "roofline_frac": round(20 * w.N * 8 * nodes / (k64 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                   "fp32_speedup": round(mlups / mlups64, 3)}
    log(f"[bench] fp64 {mlups64:.0f} MLUPS")
    d64.close()
    del d64

    # ---- FP32 vs FP64 accuracy over a short window ----
    a32 = P.Domain(precision=32, **w.params())
    a64 = P.Domain(precision=64, **w.params())
    a32.set_fields(w.c, w.u)
    a64.set_fields(w.c, w.u)
    a32.step(args.acc_steps)
    a64.step(args.acc_steps)
    err = float(np.max(np.abs(a32.get_c() - a64.get_c())))
    out["fp32_vs_fp64"] = {"steps": args.acc_steps, "max_abs_dc": err, "tolerance": 1e-5}
    log(f"[bench] fp32 vs fp64 max|dc| after {args.acc_steps} steps = {err:.3e}")
    a32.close()
    a64.close()
    del a32, a64

    if not args.no_extra:
        # ---- the other phase counts at sizes far above the 256 MB MALL ----
        sweep = []
        for name, wk in (("static_droplet_N3_4096x4096", lambda: W.static_droplet(4096, 4096, R=1000)),
                         ("droplet_collision_N4_3072x3072",
                          lambda: W.droplet_collision(3072, accept=P.accepts))):
            ww = wk()
            for prec in (32, 64):
                sweep.append(dict(workload=name, precision=f"fp{prec}",
                                  **kernel_rate(P, ww, prec, 256 if prec == 32 else 128, torch)))
                log(f"[bench] {name} fp{prec}: {sweep[-1]}")
            del ww
        out["sweep_2d"] = sweep
        # ---- force distribution of Remark 1 against eq:N20_1, same workload ----
        r1 = kernel_rate(P, w, 32, 256, torch, force_form=1)
        r1["vs_eq_N20_1_kernel_time"] = round(r1["kernel_ms"] / k_ms, 3)
        out["remark1_force"] = r1
        log(f"[bench] remark 1: {r1}")
        # ---- mixed gradient scheme (eq:N40) against the central one ----
        mx = kernel_rate(P, w, 32, 256, torch, grad_scheme=1)
        mx["vs_central_kernel_time"] = round(mx["kernel_ms"] / k_ms, 3)
        out["mixed_gradients"] = mx
        log(f"[bench] mixed gradients: {mx}")
        # ---- D3Q15 ----
        d3 = []
        for name, wk in (("static_sphere_N3_256^3", lambda: W.static_sphere(256, R=64.0)),
                         ("slabs_spheres_N5_256^3",
                          lambda: W.slabs_and_spheres(256, accept=P.accepts))):
            ww = wk()
            for prec in (32, 64):
                d3.append(dict(workload=name, precision=f"fp{prec}",
                               **kernel_rate(P, ww, prec, 128 if prec == 32 else 64, torch)))
                log(f"[bench] {name} fp{prec}: {d3[-1]}")
            del ww
        out["d3q15"] = d3

    # ---- serving: the workload table's request stream ----
    if not args.no_serving:
        log("[bench] serving run")
        import workloads as W2
        reqs = W2.request_stream(n=args.serving_requests, rate=1.0, seed=W2.BASE_SEED + 5)
        t0 = time.perf_counter()
        jobs = S._prepare(reqs, args.serving_steps_scale)
        log(f"[serving] prepared {len(jobs)} requests in {time.perf_counter() - t0:.1f} s")
        runs = []
        rate = None
        for b in args.serving_budgets.split(","):
            if b == "device":
                free, _ = torch.cuda.mem_get_info()
                budget = int(free * 0.9)
            else:
                budget = int(float(b) * (1 << 30))
            r = S.run_stream(nreq=len(jobs), steps_scale=args.serving_steps_scale, budget=budget,
                             rate=rate, jobs=jobs, log=log)
            r["budget"] = b
            rate = r["arrival_rate_per_s"]    # the same stream for every budget
            runs.append(r)
        out["serving"] = runs[0]
        if len(runs) > 1:
            out["serving_other_budgets"] = runs[1:]

    # ---- CPU oracle baseline ----
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_single_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
