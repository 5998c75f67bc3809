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


def test_sphere_256cubed_parity():
    """The D3Q15 benchmark workload (N = 3 sphere, 256^3) in the launch
    configuration the benchmark times: FP64 GPU against the 3-D oracle after
    one step, the window the oracle finishes in seconds at this size."""
    from oracle import OracleSim3D
    w = W.static_sphere(256, R=64.0)
    print(f"case {w.name} 256^3 steps=1", flush=True)
    o = OracleSim3D(**w.params())
    o.init(w.c, w.u)
    o.step(1)
    d = gpu_domain(w, precision=64)
    d.step(1)
    for a, b in zip(d.macro(), o.macro()):
        assert maxabs(a, b) < TOL
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
