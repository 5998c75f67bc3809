"""Parity at the full sizes of the workload table, in the launch
configuration the benchmark times (single-domain strip decomposition):
FP64 GPU vs the FP64 oracle over windows the oracle finishes in seconds,
and FP32 vs FP64 on the benchmark workload (N=5, 2048x2048)."""
import numpy as np
import pytest

import workloads as W
from oracle.accept import oracle_accepts
from tests.gpu_util import gpu_domain, maxabs, oracle_run

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _check(w, steps):
    print(f"case {w.name} {w.nx}x{w.ny} N={w.N} steps={steps}", flush=True)
    o = oracle_run(w, steps)
    d = gpu_domain(w, precision=64)
    d.step(steps)
    for a, b in zip(d.macro(), o.macro()):
        assert maxabs(a, b) < TOL


def test_lens_400x200_parity():
    _check(W.liquid_lens(s12=1e-3, s13=1.4e-3, s23=0.6e-3), 400)


def test_collision_512_parity():
    _check(W.droplet_collision(512, accept=oracle_accepts, precision=64), 40)


def test_bands_2048_parity():
    _check(W.bands_and_droplets(2048, accept=oracle_accepts, precision=64), 2)


def test_bands_2048_fp32_vs_fp64():
    w = W.bands_and_droplets(2048, accept=oracle_accepts)
    d32 = gpu_domain(w, precision=32)
    d64 = gpu_domain(w, precision=64)
    d32.step(200)
    d64.step(200)
    assert np.max(np.abs(d32.get_c() - d64.get_c())) < 1e-5
    m0 = d64.diagnostics()[0]
    assert np.all(np.isfinite(m0))


@pytest.mark.timeout(900)
@pytest.mark.parametrize("which,checkpoints", [("sphere", [1, 20, 60]), ("slabs", [8, 24])])
def test_256cubed_parity(which, checkpoints):
    """The D3Q15 benchmark workloads (the N = 3 sphere and the N = 5 slabs
    and spheres, 256^3) in the launch configuration the benchmark times:
    FP64 GPU against the 3-D oracle after 1, 20 and 60 steps (sphere; the
    runs replay graphs of 16 and 4, 32 and 8 steps) and 8 and 24 steps
    (slabs), windows the oracle finishes in about a minute each at this
    size on 16 host threads."""
    from oracle import OracleSim3D
    w = (W.static_sphere(256, R=64.0) if which == "sphere"
         else W.slabs_and_spheres(256, accept=oracle_accepts))
    o = OracleSim3D(**w.params())
    o.init(w.c, w.u)
    d = gpu_domain(w, precision=64)
    t = 0
    for cp in checkpoints:
        print(f"case {w.name} 256^3 N={w.N} steps={cp}", flush=True)
        o.step(cp - t)
        d.step(cp - t)
        t = cp
        err = max(maxabs(a, b) for a, b in zip(d.macro(), o.macro()))
        print(f"  t={t}: max |GPU - oracle| = {err:.2e}", flush=True)
        assert err < TOL
    d.close()


def test_slabs_256cubed_fp32_vs_fp64():
    w = W.slabs_and_spheres(256, accept=oracle_accepts)
    d32 = gpu_domain(w, precision=32)
    d64 = gpu_domain(w, precision=64)
    d32.step(100)
    d64.step(100)
    assert np.max(np.abs(d32.get_c() - d64.get_c())) < 1e-5
    m, dev, bad = d32.diagnostics()
    assert bad == 0 and dev < 1e-5


@pytest.mark.parametrize("which,steps", [("collision", 50000), ("bands", 20000)])
def test_fp32_vs_fp64_over_the_whole_run(which, steps):
    """The FP32 mode within 1e-5 of the FP64 mode on every c_i over the
    whole run of the N = 4 droplet collision (512^2, 50000 steps, droplets
    moving at 0.01) and the N = 5 bands-and-droplets layout (2048^2, 20000
    steps), checked every 10000 steps, with per-phase mass conserved.  The
    moving droplets are the hard case: an FP32 evaluation of the NS
    collision gave them a steady momentum bias (2.6e-5 after 2000 steps,
    2e-3 after 50000)."""
    if which == "collision":
        w = W.droplet_collision(512, accept=oracle_accepts)
    else:
        w = W.bands_and_droplets(2048, accept=oracle_accepts)
    print(f"case {w.name} {w.nx}x{w.ny} fp32 vs fp64 steps={steps}", flush=True)
    d32 = gpu_domain(w, precision=32)
    d64 = gpu_domain(w, precision=64)
    m0 = d32.diagnostics()[0]
    done = 0
    while done < steps:
        n = min(10000, steps - done)
        d32.step(n)
        d64.step(n)
        done += n
        err = maxabs(d32.get_c(), d64.get_c())
        print(f"  t={done}: max|c32 - c64| = {err:.2e}", flush=True)
        assert err < 1e-5
    m1, dev, bad = d32.diagnostics()
    d32.close()
    d64.close()
    assert bad == 0 and dev < 1e-6
    assert np.max(np.abs(m1 - m0) / m0) < 1e-8
