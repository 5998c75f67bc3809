"""FP64 parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerance: 1e-10 max-abs on c, u and p (the stated FP64 bar).  Inputs are
seeded and synthetic (workloads module); sizes span several strips of the
marching kernel (48 interior columns in FP64, 16+ rows) with ragged last
strips in x and y, both boundary kinds, N = 2..5, spatially varying tau_g (unequal
mu/rho), a body force, and the graph path (>= 64 steps).
"""
import numpy as np
import pytest

import workloads as W
from oracle.accept import oracle_accepts
from tests.gpu_util import gpu_domain, maxabs, oracle_run

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.mark.parametrize("N", [2, 3, 4, 5])
@pytest.mark.parametrize("wall", [False, True])
def test_random_parity(N, wall):
    w = W.random_smooth(N, 130, 70, seed=100 + N + 10 * wall, wall_y=wall, accept=oracle_accepts)
    steps = 40
    print(f"case random N={N} wall={wall} 130x70 steps={steps}", flush=True)
    o = oracle_run(w, steps)
    d = gpu_domain(w)
    d.step(steps)
    co, uo, po = o.macro()
    cg, ug, pg = d.macro()
    assert d.time == steps
    assert maxabs(cg, co) < TOL
    assert maxabs(ug, uo) < TOL
    assert maxabs(pg, po) < TOL


def test_tiny_domain_parity():
    # nx, ny smaller than one strip: lanes wrap around the periodic domain
    w = W.random_smooth(3, 12, 10, seed=7, wall_y=False, accept=oracle_accepts)
    o = oracle_run(w, 30)
    d = gpu_domain(w)
    d.step(30)
    for a, b in zip(d.macro(), o.macro()):
        assert maxabs(a, b) < TOL


def test_tiny_wall_parity():
    w = W.random_smooth(4, 9, 4, seed=8, wall_y=True, accept=oracle_accepts)
    o = oracle_run(w, 30)
    d = gpu_domain(w)
    d.step(30)
    for a, b in zip(d.macro(), o.macro()):
        assert maxabs(a, b) < TOL


def test_static_droplet_parity_graph_path():
    # configuration 1 layout (N=3, 100x100, R=25), 130 steps: two graph
    # replays of 64 steps plus eager steps
    w = W.static_droplet()
    o = oracle_run(w, 130)
    d = gpu_domain(w)
    d.step(130)
    for a, b in zip(d.macro(), o.macro()):
        assert maxabs(a, b) < TOL


def test_lens_parity():
    # configuration 2 layout (N=3, 400x200, walls in y), unequal tensions
    w = W.liquid_lens(s12=1e-3, s13=0.8e-3, s23=1.2e-3)
    o = oracle_run(w, 60)
    d = gpu_domain(w)
    d.step(60)
    for a, b in zip(d.macro(), o.macro()):
        assert maxabs(a, b) < TOL


def test_diagnostics_and_laplace_match_oracle():
    w = W.static_droplet()
    o = oracle_run(w, 50)
    d = gpu_domain(w)
    d.step(50)
    mass, dev, bad = d.diagnostics()
    assert np.allclose(mass, o.mass(), rtol=0, atol=1e-9)
    c, u, p = o.macro()
    assert dev == pytest.approx(np.max(np.abs(c.sum(0) - 1.0)), abs=1e-14)
    assert bad == 0
    y, x = np.mgrid[0:100, 0:100]
    r = np.hypot(x - 50.0, y - 50.0)
    ref = p[r <= 17].mean() - p[r >= 33].mean()
    assert d.laplace(50.0, 50.0, 17.0, 33.0) == pytest.approx(ref, abs=1e-12)


def test_determinism_and_checkpoint():
    w = W.random_smooth(3, 70, 40, seed=3, accept=oracle_accepts)
    d1 = gpu_domain(w)
    d1.step(20)
    st, t = d1.get_state()
    d1.step(21)
    d2 = gpu_domain(w)
    d2.set_state(st, t)
    d2.step(21)
    assert d2.time == d1.time == 41
    for a, b in zip(d1.macro(), d2.macro()):
        assert np.array_equal(a, b)
