"""Body force and walls on the HIP path (FP64): parity with the oracle on
the gravity workloads of Sec. 4.2 (floating puddle) and Sec. 4.3 (four-phase
droplet and bubble, eq:N38), the puddle thickness against de Gennes' balance
(eq:N37 extended to a heavy upper phase), and the surface-tension effect on
the falling droplet that Sec. 4.3 reports.

Measured on MI355X: puddle R = 40 on 600 x 200, g = 2e-5: H = 28.88 against
28.87; g = 5e-5: 18.73 against 18.26; at g = 2e-5 with sigma_13 = 0.006, 0.008,
0.012, 0.014 (sigma_12 = sigma_23 = 0.01): 22.78, 26.0, 31.6, 34.1 against
22.36, 25.82, 31.62, 34.16 after 300 000 steps.  Four-phase run to t = 12.25 (time
unit sqrt(D / g)): mean droplet speed over t = 6.5 .. 12.25 is 0.365 sqrt(gD)
for sigma_13 = 0.01 and 0.313 for sigma_13 = 0.006."""
import numpy as np
import pytest

import workloads as W
from physics_util import centroid_velocity, de_gennes_thickness, puddle_thickness
from tests.gpu_util import gpu_domain, maxabs, oracle_run

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.mark.parametrize("name", ["puddle", "four_phase"])
def test_gravity_workload_parity(name):
    if name == "puddle":
        w = W.floating_puddle(200, 100, R=20.0, g=1e-4)
        steps = 80
    else:
        w = W.four_phase_buoyancy()
        steps = 60
    print(f"case {w.name} {w.nx}x{w.ny} steps={steps}", flush=True)
    o = oracle_run(w, steps)
    d = gpu_domain(w)
    d.step(steps)
    for a, b in zip(d.macro(), o.macro()):
        assert maxabs(a, b) < TOL
    d.close()


def test_puddle_thickness_de_gennes():
    """Large puddles (R = 40 on 600 x 200, rho = 3 : 1 : 6, sigma = 0.01):
    the thickness tends to the de Gennes value; H ~ g^(-1/2)."""
    H = {}
    for g, tol in ((2e-5, 0.02), (5e-5, 0.04)):
        w = W.floating_puddle(600, 200, R=40.0, g=g)
        d = gpu_domain(w)
        d.step(300_000)
        _, _, bad = d.diagnostics()
        H[g] = puddle_thickness(d.get_c())
        d.close()
        assert bad == 0
        Hth = de_gennes_thickness(0.01, 0.01, 0.01, 3.0, 1.0, 6.0, g)
        print(f"g={g} H={H[g]:.3f} de Gennes {Hth:.3f}", flush=True)
        assert abs(H[g] - Hth) / Hth < tol
    assert H[2e-5] / H[5e-5] == pytest.approx(np.sqrt(5 / 2), rel=0.03)


def test_four_phase_droplet_falls_slower_with_lower_tension():
    """Sec. 4.3: the phase-1 droplet falls and the phase-2 bubble rises; with
    sigma_13 = 0.006 (Bo = 18) the droplet deforms more and falls slower than
    with sigma_13 = 0.01 (Bo = 10.8)."""
    Us = np.sqrt(1e-5 * 60.0)
    speed = {}
    for s13 in (0.01, 0.006):
        w = W.four_phase_buoyancy(sigma13=s13)
        d = gpu_domain(w)
        late = []
        for k in range(15):
            d.step(2000)
            c, u, _ = d.macro()
            v1 = centroid_velocity(c, u, 0)[1] / Us
            v2 = centroid_velocity(c, u, 1)[1] / Us
            if k < 4:
                assert v1 < 0 < v2     # droplet down, bubble up
            if k >= 7:
                late.append(-v1)
        d.close()
        speed[s13] = np.mean(late)
        print(f"sigma_13={s13}: mean late fall speed {speed[s13]:.3f}", flush=True)
    assert speed[0.006] < 0.95 * speed[0.01]


def test_puddle_thickness_against_sigma13():
    """H(sigma_13) at g = 2e-5 (R = 40 on 600 x 200, rho = 3 : 1 : 6,
    sigma_12 = sigma_23 = 0.01): de Gennes' balance (eq:N37 with the upper
    phase's density kept) gives H^2 proportional to the spreading term
    sigma_12 + sigma_13 - sigma_23 = sigma_13."""
    H = {}
    for s13, tol in ((0.006, 0.03), (0.014, 0.02)):
        w = W.floating_puddle(600, 200, R=40.0, g=2e-5, sigma=(0.01, s13, 0.01))
        print(f"case puddle sigma_13={s13} 600x200 steps=300000", flush=True)
        d = gpu_domain(w)
        d.step(300_000)
        _, _, bad = d.diagnostics()
        H[s13] = puddle_thickness(d.get_c())
        d.close()
        assert bad == 0
        Hth = de_gennes_thickness(0.01, s13, 0.01, 3.0, 1.0, 6.0, 2e-5)
        print(f"  H={H[s13]:.3f} de Gennes {Hth:.3f}", flush=True)
        assert abs(H[s13] - Hth) / Hth < tol
    assert H[0.014] / H[0.006] == pytest.approx(np.sqrt(0.014 / 0.006), rel=0.03)
