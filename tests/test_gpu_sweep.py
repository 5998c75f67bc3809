"""A seeded sweep over the parameter space of the 2-D step, FP64 on the HIP
path against the oracle (1e-10 max-abs on c, u, p): phase counts 2..8, the
three schemes, periodic or walls, lattice sides from below one strip to
several strips with ragged tails, interface widths 3..6, random tensions,
densities, viscosities (tau_g varying in space), mobilities, tau_phi and
body forces.  Each case is drawn from its own seed, so a failure names a
reproducible case."""
import numpy as np
import pytest

import workloads as W
from oracle.accept import oracle_accepts
from tests.gpu_util import gpu_domain, maxabs, oracle_run

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _case(seed):
    rng = np.random.default_rng(7000 + seed)
    N = int(rng.integers(2, 9))
    scheme = ["central", "mixed", "remark1"][int(rng.integers(0, 3))]
    nx = int(rng.choice([5, 9, 17, 40, 63, 100, 131, 230, 257]))
    ny = int(rng.choice([4, 6, 11, 33, 70]))
    wall = bool(rng.integers(0, 2))
    Wd = float(rng.uniform(3.0, 6.0))
    sig = (0.5e-3, 2e-3) if N <= 5 else (0.8e-3, 1.2e-3)
    w = W.random_smooth(N, nx, ny, seed=8000 + seed, wall_y=wall, accept=oracle_accepts, W=Wd,
                        sigma_range=sig)
    over = {"central": {}, "mixed": {"grad_scheme": 1}, "remark1": {"force_form": 1}}[scheme]
    return w, over, f"N={N} {scheme} {nx}x{ny} wall={wall} W={Wd:.2f}"


@pytest.mark.parametrize("seed", range(24))
def test_seeded_parameter_sweep(seed):
    w, over, name = _case(seed)
    steps = 25
    print(f"case seed={seed} {name} steps={steps}", flush=True)
    o = oracle_run(w, steps, **over)
    d = gpu_domain(w, **over)
    d.step(steps)
    res = [maxabs(a, b) for a, b in zip(d.macro(), o.macro())]
    d.close()
    assert max(res) < TOL, (name, res)
