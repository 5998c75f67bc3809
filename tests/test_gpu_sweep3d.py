"""A seeded sweep over the D3Q15 step, FP64 on the HIP path against the 3-D
oracle (1e-10 max-abs on c, u, p): N = 2..5, periodic or walls in z, and
plane counts of the form 8 k + 1 (with 8-plane segments the last segment
is one plane, and the segment below it marches down from one plane inside
the wall), besides others; x and y sizes below and above one tile."""
import numpy as np
import pytest

import workloads as W
from oracle import OracleSim3D
from oracle.accept import oracle_accepts
from tests.gpu_util import gpu_domain, maxabs

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _case(seed):
    rng = np.random.default_rng(9000 + seed)
    N = int(rng.integers(2, 6))
    nx = int(rng.choice([6, 23, 64, 70]))
    ny = int(rng.choice([4, 7, 13]))
    nz = int(rng.choice([5, 9, 12, 17, 25]))
    wall = bool(rng.integers(0, 2)) or nz in (9, 17, 25)
    w = W.random_smooth3d(N, nx, ny, nz, seed=9500 + seed, wall_z=wall, accept=oracle_accepts)
    return w, f"N={N} {nx}x{ny}x{nz} wall={wall}"


@pytest.mark.parametrize("seed", range(12))
def test_seeded_3d_sweep(seed):
    w, name = _case(seed)
    steps = 12
    print(f"case seed={seed} {name} steps={steps}", flush=True)
    o = OracleSim3D(**w.params())
    o.init(w.c, w.u)
    o.step(steps)
    d = gpu_domain(w)
    d.step(steps)
    res = [maxabs(a, b) for a, b in zip(d.macro(), o.macro())]
    d.close()
    assert max(res) < TOL, (name, res)
