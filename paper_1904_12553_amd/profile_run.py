"""Small driver for rocprofv3 runs (kernel traces and HBM counters).

    python3 -m paper_1904_12553_amd.profile_run --what step --steps 10
    python3 -m paper_1904_12553_amd.profile_run --what step3d --n3 5 --steps 10
    python3 -m paper_1904_12553_amd.profile_run --what copy --mib 1024
    python3 -m paper_1904_12553_amd.profile_run --what sweep --n2 3 --steps 10

``step`` runs the benchmark workload (N=5, 2048 x 2048, FP32, the same
launch configuration as bench.py) for a few eager steps; ``step3d`` the
D3Q15 workloads of the benchmark (256^3, N = 5 slabs and spheres or the
N = 3 static sphere) or, with ``--n3 4``, three moving spheres at 192^3;
``sweep`` the other 2-D phase counts of the benchmark (``--n2 3``: the
N = 3 static droplet at 4096^2, ``--n2 4``: the N = 4 droplet collision at
3072^2); ``copy`` runs the
library's plain copy kernel over a buffer of known size, whose FETCH_SIZE /
WRITE_SIZE readings calibrate the counters, and prints the copy bandwidth
measured with HIP events.
"""
import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--what", choices=["step", "step3d", "sweep", "copy"], default="step")
    ap.add_argument("--n2", type=int, default=3, choices=[3, 4],
                    help="phases of the 2-D sweep workload")
    ap.add_argument("--n3", type=int, default=5, choices=[3, 4, 5],
                    help="phases of the 3-D workload")
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--side", type=int, default=2048)
    ap.add_argument("--precision", type=int, default=32)
    ap.add_argument("--scheme", choices=["central", "mixed", "remark1"], default="central",
                    help="2-D step kernel: eq:N31a, eq:N40 gradients, or Remark 1's force")
    ap.add_argument("--mib", type=int, default=1024)
    args = ap.parse_args()
    import torch
    import paper_1904_12553_amd as P
    import workloads as W
    torch.cuda.set_device(0)
    if args.what == "copy":
        n = args.mib << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda")
        b = torch.empty(n, dtype=torch.uint8, device="cuda")
        a.fill_(1)
        for _ in range(3):
            P.device_copy(b, a, n)
        torch.cuda.synchronize()
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        e0.record(st)
        for _ in range(reps):
            P.device_copy(b, a, n)
        e1.record(st)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        print(json.dumps({"copy_bytes": n, "ms": ms, "GBps_read_plus_write": 2 * n / ms / 1e6}))
        return
    if args.what == "sweep":
        w = (W.static_droplet(4096, 4096, R=1000) if args.n2 == 3
             else W.droplet_collision(3072, accept=P.accepts))
    elif args.what == "step3d":
        w = {5: lambda: W.slabs_and_spheres(256, accept=P.accepts),
             4: lambda: W.droplet_collision3d(192, accept=P.accepts),
             3: lambda: W.static_sphere(256, R=64.0)}[args.n3]()
    else:
        w = W.bands_and_droplets(args.side, accept=P.accepts)
    over = {"central": {}, "mixed": {"grad_scheme": 1}, "remark1": {"force_form": 1}}[args.scheme]
    d = P.Domain(precision=args.precision, **dict(w.params(), **over))
    d.set_fields(w.c, w.u)
    os.environ["NPLBM_NO_GRAPH"] = "1"
    d.step(args.steps)
    d.sync()
    print(json.dumps({"steps": args.steps, "nodes": d.n, "N": w.N,
                      "precision": args.precision}))


if __name__ == "__main__":
    main()
