"""Parity over the full windows of the workload table, in the launch
configuration the benchmark times (single-domain strip decomposition, the
graph path for runs of 64 steps and more):

- the static droplet (N = 3, 100 x 100, Sec. 4.1 set-up): all 2000 steps;
- the liquid lens (N = 3, 400 x 200, walls, Sec. 4.2 set-up) on a diagonal
  tension case (sigma_13 = sigma_23): all 20 000 steps;
- the droplet collision (N = 4, 512^2): the first 2000 steps;
- the bands and droplets (N = 5, 2048^2, the benchmark workload): the first
  200 steps.

FP64 GPU against the FP64 oracle at 1e-10 max-abs on c, u and p, checked at
several points of each window; the FP32 mode against the FP64 mode at
1e-5 max-abs on every c_i at the end of each window (the lens at 20 000
steps), and the Laplace jump of the droplet within 0.5%.  The oracle runs
on all host cores; these windows cost it about 3 minutes in total.
"""
import numpy as np
import pytest

import workloads as W
from oracle.accept import oracle_accepts
from tests.gpu_util import gpu_domain, maxabs, oracle_run

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]
TOL = 1e-10


def _window(w, checkpoints, fp32=True):
    from oracle import OracleSim
    print(f"case window {w.name} {w.nx}x{w.ny} N={w.N} to t={checkpoints[-1]}", flush=True)
    o = OracleSim(**w.params())
    o.init(w.c, w.u)
    d = gpu_domain(w, precision=64)
    t = 0
    for cp in checkpoints:
        o.step(cp - t)
        d.step(cp - t)
        t = cp
        err = max(maxabs(a, b) for a, b in zip(d.macro(), o.macro()))
        print(f"  t={t}: max |GPU - oracle| = {err:.2e}", flush=True)
        assert err < TOL, (w.name, t, err)
    if fp32:
        d32 = gpu_domain(w, precision=32)
        d32.step(t)
        e32 = maxabs(d32.get_c(), d.get_c())
        print(f"  t={t}: max |c32 - c64| = {e32:.2e}", flush=True)
        assert e32 < 1e-5
        return d, d32
    return d, None


def test_static_droplet_full_window():
    w = W.static_droplet()
    d, d32 = _window(w, [500, 1000, 2000])
    # Laplace jump (bulk means inside R - 2W and outside R + 2W), FP32 vs FP64
    dp64 = d.laplace(50.0, 50.0, 17.0, 33.0)
    dp32 = d32.laplace(50.0, 50.0, 17.0, 33.0)
    assert dp64 > 0
    assert abs(dp32 - dp64) / dp64 < 5e-3


def test_lens_diagonal_tensions_full_window():
    w = W.liquid_lens(s12=1e-3, s13=0.8e-3, s23=0.8e-3)
    _window(w, [2000, 5000, 10000, 20000])


def test_collision_512_first_2000_steps():
    _window(W.droplet_collision(512, accept=oracle_accepts, precision=64), [500, 2000])


def test_bands_2048_first_200_steps():
    _window(W.bands_and_droplets(2048, accept=oracle_accepts, precision=64), [64, 200])
