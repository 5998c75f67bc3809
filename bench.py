"""Benchmark of the fused N-phase LB step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-serving]

Workload (one "step" = one pass of the whole hot path): the N=5 droplets and
interfaces configuration -- 2048 x 2048 periodic lattice, four stacked bands
of phases 1-4 plus 64 seeded phase-5 droplets (r ~ U[10, 40]), sigma_kl ~
U[0.5e-3, 2e-3] (SPD-checked), rho_k ~ U[1, 3], FP32 state -- advanced by
the fused step kernel, with the FP64 conservation diagnostics (per-phase
mass, max |sum c - 1|, non-finite count) every 100 steps inside the timed
region.  Inputs are resident in HBM before timing starts.

Prints ONE JSON line: MLUPS (node updates per second / 1e6), the roofline
object of the step kernel (algorithmic bytes 20 N s per node update over the
kernel's average duration, measured with HIP events on the stream the kernel
runs on), the FP64 run of the same workload and its speedup, the FP32-vs-FP64
error on c after a short window, mass drift, a serving run (p50/p99
time-to-completion and aggregate MLUPS) and the FP64 CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
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


def traffic_from_profiles(nodes, steps_unit="launch"):
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


def time_steps(d, steps, torch, stream, diag_every=DIAG_EVERY):
    """Run `steps` steps with diagnostics every `diag_every`; returns
    (wall seconds, summed step-kernel seconds from events, last diag)."""
    ev = []
    diag = None
    done = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while done < steps:
        n = min(diag_every, steps - done)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        d.step(n)
        b.record(stream)
        ev.append((a, b, n))
        done += n
        if done % diag_every == 0:
            diag = d.diagnostics()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern = sum(a.elapsed_time(b) for a, b, _ in ev) / 1e3
    return wall, kern, diag


def kernel_rate(P, w, prec, steps, torch, stream, **over):
    """Step-kernel time of a workload (HIP events around `steps` steps after
    a warmup): ms per step, MLUPS and the fraction of the HBM roofline with
    the algorithmic bytes per node update -- 20 N s on D2Q9, 2 (16 N + 1) s
    on D3Q15 -- for state word size s."""
    d = P.Domain(precision=prec, **dict(w.params(), **over))
    d.set_fields(w.c, w.u)
    d.step(64)
    d.sync()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    d.step(steps)
    b.record(stream)
    b.synchronize()
    ms = a.elapsed_time(b) / steps
    nodes = d.n
    s = 8 if prec == 64 else 4
    B = (2 * (16 * w.N + 1) if d.dim == 3 else 20 * w.N) * s
    d.close()
    return {"kernel_ms": round(ms, 5), "MLUPS": round(nodes / ms / 1e3, 1),
            "bytes_per_node_update": B,
            "roofline_frac": round(nodes * B / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--side", type=int, default=2048)
    ap.add_argument("--fp64-steps", type=int, default=500)
    ap.add_argument("--acc-steps", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=40)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=96)
    ap.add_argument("--serving-steps-scale", type=float, default=0.1)
    ap.add_argument("--profile-only", action="store_true",
                    help="only the warmup and timed FP32 steps (for rocprofv3 runs)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the N = 3 / 4 sweep, the Remark 1 and the D3Q15 legs")
    args = ap.parse_args()

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
    stream = torch.cuda.current_stream()
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
    wall, kern, diag = time_steps(d, args.steps, torch, stream)
    mlups = nodes * args.steps / wall / 1e6
    ms_step = wall / args.steps * 1e3
    k_ms = kern / args.steps * 1e3
    achieved = B_node * nodes / (k_ms * 1e-3) / 1e9
    log(f"[bench] fp32 {mlups:.0f} MLUPS, {ms_step:.4f} ms/step, kernel {k_ms:.4f} ms, "
        f"{achieved:.0f} GB/s")
    mass_T = diag[0] if diag is not None else d.diagnostics()[0]
    drift = float(np.max(np.abs(mass_T - m0) / np.abs(m0)))
    if args.profile_only:
        print(json.dumps({"metric": "MLUPS", "value": round(mlups, 1), "profile_only": True}))
        return
    d.close()
    del d

    out = {
        "metric": "MLUPS (N=5, FP32, fused step incl. FP64 diagnostics every 100 steps)",
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
                   "diag_every": DIAG_EVERY},
    }
    traffic = traffic_from_profiles(nodes)
    out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                       "traffic": traffic,
                       "bytes_per_node_update": B_node, "kernel_ms": round(k_ms, 5)}
    out["mass_drift_rel"] = drift

    # ---- FP64 run of the same workload ----
    d64 = P.Domain(precision=64, **w.params())
    d64.set_fields(w.c, w.u)
    d64.step(args.warmup)
    wall64, kern64, _ = time_steps(d64, args.fp64_steps, torch, stream)
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
                                  **kernel_rate(P, ww, prec, 200 if prec == 32 else 100, torch,
                                                stream)))
                log(f"[bench] {name} fp{prec}: {sweep[-1]}")
            del ww
        out["sweep_2d"] = sweep
        # ---- force distribution of Remark 1 against eq:N20_1, same workload ----
        r1 = kernel_rate(P, w, 32, 300, torch, stream, force_form=1)
        r1["vs_eq_N20_1_kernel_time"] = round(r1["kernel_ms"] / k_ms, 3)
        out["remark1_force"] = r1
        log(f"[bench] remark 1: {r1}")
        # ---- D3Q15 ----
        d3 = []
        for name, wk in (("static_sphere_N3_256^3", lambda: W.static_sphere(256, R=64.0)),
                         ("slabs_spheres_N5_256^3",
                          lambda: W.slabs_and_spheres(256, accept=P.accepts))):
            ww = wk()
            for prec in (32, 64):
                d3.append(dict(workload=name, precision=f"fp{prec}",
                               **kernel_rate(P, ww, prec, 100 if prec == 32 else 50, torch,
                                             stream)))
                log(f"[bench] {name} fp{prec}: {d3[-1]}")
            del ww
        out["d3q15"] = d3

    # ---- serving ----
    if not args.no_serving:
        log("[bench] serving run")
        out["serving"] = S.run_stream(nreq=args.serving_requests,
                                      steps_scale=args.serving_steps_scale, log=log)

    # ---- CPU oracle baseline ----
    if not args.no_cpu:
        from oracle import OracleSim
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        log(f"[bench] cpu oracle sample: {args.cpu_steps} steps of the same workload, "
            f"{threads} threads")
        o = OracleSim(**w.params())
        o.init(w.c, w.u)
        t0 = time.perf_counter()
        o.step(args.cpu_steps)
        ct = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(nodes * args.cpu_steps / ct / 1e6, 4),
                               "unit": "MLUPS", "cores": threads, "kind": "oracle",
                               "sample": f"{args.cpu_steps} FP64 steps of the {side}x{side} N=5 "
                                         f"workload ({ct:.1f} s)"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
