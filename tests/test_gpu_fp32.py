"""FP32 mode (deviation storage: g_1..g_8 only, h_0 rebuilt from phi) against
the GPU FP64 mode: 1e-5 max-abs on every c_i, Laplace pressure within 0.5%,
per-phase mass conserved to FP32 round-off."""
import numpy as np
import pytest

import workloads as W
from oracle.accept import oracle_accepts
from tests.gpu_util import gpu_domain

pytestmark = pytest.mark.gpu


def test_static_droplet_fp32_vs_fp64_and_laplace():
    # static droplet configuration: N=3, 100x100, R=25, sigma=1e-3, 2000 steps
    w = W.static_droplet()
    d32 = gpu_domain(w, precision=32)
    d64 = gpu_domain(w, precision=64)
    m32 = d32.diagnostics()[0]
    # Laplace pressure averaged over the last 500 steps (acoustic waves)
    d32.step(1500)
    d64.step(1500)
    dp32, dp64 = [], []
    for _ in range(50):
        d32.step(10)
        d64.step(10)
        dp32.append(d32.laplace(50.0, 50.0, 25.0 - 8.0, 25.0 + 8.0))
        dp64.append(d64.laplace(50.0, 50.0, 25.0 - 8.0, 25.0 + 8.0))
    assert d32.time == 2000
    c32, c64 = d32.get_c(), d64.get_c()
    assert np.max(np.abs(c32 - c64)) < 1e-5
    a32, a64 = np.mean(dp32), np.mean(dp64)
    assert abs(a32 - a64) <= 0.005 * abs(a64)
    mass, dev, bad = d32.diagnostics()
    assert bad == 0
    assert np.max(np.abs(mass - m32) / np.abs(m32).max()) < 1e-5


@pytest.mark.parametrize("N,wall", [(3, True), (4, False), (5, True), (5, False)])
def test_random_fp32_vs_fp64(N, wall):
    w = W.random_smooth(N, 190, 100, seed=300 + N + wall, wall_y=wall, accept=oracle_accepts,
                        amp_u=5e-3)
    d32 = gpu_domain(w, precision=32)
    d64 = gpu_domain(w, precision=64)
    d32.step(1000)
    d64.step(1000)
    assert np.max(np.abs(d32.get_c() - d64.get_c())) < 1e-5
    assert np.max(np.abs(d32.get_u() - d64.get_u())) < 1e-6


def test_moving_droplets_fp32_gap_does_not_grow():
    """The N = 4 collision layout at 256^2 (droplets moving at 0.01): the
    FP32 - FP64 gap on c after 4000 steps is within 1e-5 and no more than
    four times the gap after 1000 steps (with the NS collision evaluated in
    FP32 arithmetic it grew as t^2)."""
    w = W.droplet_collision(256, accept=oracle_accepts)
    print(f"case {w.name} 256^2 fp32 vs fp64 steps=4000", flush=True)
    a = gpu_domain(w, precision=64)
    b = gpu_domain(w, precision=32)
    a.step(1000)
    b.step(1000)
    e1 = float(np.max(np.abs(a.get_c() - b.get_c())))
    a.step(3000)
    b.step(3000)
    e4 = float(np.max(np.abs(a.get_c() - b.get_c())))
    a.close()
    b.close()
    print(f"  |c32 - c64|: {e1:.2e} after 1000 steps, {e4:.2e} after 4000", flush=True)
    assert e4 < 1e-5
    assert e4 < 4 * e1 + 1e-7
