"""CPU pins of the lens measures used by the physics tests (Sec. 4.2):
eq:N32 angles, eq:N33 area / length relation, eq:N34 cap heights, against
the values Table 2 prints, closed forms and a synthetic lens of known
shape."""
import json
import os

import numpy as np
import pytest

from physics_util import (de_gennes_thickness, lens_geometry, lens_shape, neumann_angles,
                          puddle_thickness)

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "lens_table2.json")))


def _area(d, t1, t2):
    th = np.radians([t1, t2])
    return (d / 2) ** 2 * np.sum((th / np.sin(th) - np.cos(th)) / np.sin(th))   # eq:N33


@pytest.mark.parametrize("case", GOLD["cases"])
def test_table2_heights_follow_from_d_and_angles(case):
    t1, t2 = neumann_angles(*case["sigma"])
    A = _area(case["d"], t1, t2)
    d, h1, h2 = lens_shape(A, t1, t2)
    tol = GOLD["printed_digits"] + 1e-9
    assert d == pytest.approx(case["d"], abs=1e-9)
    assert abs(h1 - case["h1"]) <= tol and abs(h2 - case["h2"]) <= tol


def test_neumann_closed_forms():
    # equal tensions: 60 degrees; the angles of the force triangle obey the
    # law of sines, sigma_12 sin(theta_1) = sigma_13 sin(theta_2)
    assert neumann_angles(1, 1, 1) == pytest.approx((60.0, 60.0))
    s12, s13, s23 = 1.0, 4 / 3, 1.0
    t1, t2 = np.radians(neumann_angles(s12, s13, s23))
    assert s12 * np.sin(t1) == pytest.approx(s13 * np.sin(t2))
    assert s12 * np.cos(t1) + s13 * np.cos(t2) == pytest.approx(s23)


def test_half_disc_lens_is_measured_exactly():
    """A lens of two circular caps with 90-degree angles (two half discs of
    radius r) has d = 2r, h_1 = h_2 = r, A = pi r^2; the measure on a sharp
    field with a linear ramp recovers them to a fraction of a lattice unit."""
    nx, ny, r = 200, 160, 40.0
    y0 = 80.3
    x, y = np.meshgrid(np.arange(nx, dtype=float), np.arange(ny, dtype=float))
    dist = np.hypot(x - 100.0, y - y0)
    c1 = np.clip(0.5 + (r - dist) / 4.0, 0.0, 1.0)
    top = np.clip(0.5 + (y - y0) / 4.0, 0.0, 1.0)
    c2 = np.clip(top - c1, 0.0, 1.0)
    c = np.stack([c1, c2, 1.0 - c1 - c2])
    g = lens_geometry(c)
    assert g["d"] == pytest.approx(2 * r, abs=0.3)
    assert g["h1"] == pytest.approx(r, abs=0.3) and g["h2"] == pytest.approx(r, abs=0.3)
    assert g["theta1"] == pytest.approx(90.0, abs=0.5)
    assert g["A"] == pytest.approx(np.pi * r * r, rel=0.01)
    d, h1, h2 = lens_shape(np.pi * r * r, 90.0, 90.0)
    assert (d, h1, h2) == pytest.approx((2 * r, r, r))


def test_de_gennes_thickness_reduces_to_eq_N37():
    # eq:N37 is the light-upper-phase limit rho_2 -> 0
    s, g = 0.01, 1e-4
    rho1, rho3 = 3.0, 6.0
    eq37 = np.sqrt(2 * (s + s - s) / ((rho1 / rho3) * (rho3 - rho1) * g))
    assert de_gennes_thickness(s, s, s, rho1, 0.0, rho3, g) == pytest.approx(eq37, rel=1e-14)
    # a heavier upper phase makes the puddle thicker; H scales as g^(-1/2)
    assert de_gennes_thickness(s, s, s, rho1, 1.0, rho3, g) > eq37
    assert (de_gennes_thickness(s, s, s, 3, 1, 6, g) / de_gennes_thickness(s, s, s, 3, 1, 6, 4 * g)
            == pytest.approx(2.0))


def test_puddle_thickness_measure():
    # a flat slab of phase 1 with linear ramps: thickness between crossings
    ny, nx = 60, 50
    y = np.arange(ny, dtype=float)[:, None] * np.ones((1, nx))
    c1 = np.clip(np.minimum(y - 20.3, 35.8 - y) / 3.0 + 0.5, 0.0, 1.0)
    c = np.stack([c1, 1 - c1, np.zeros_like(c1)])
    assert puddle_thickness(c) == pytest.approx(15.5, abs=1e-9)


def test_line_tension_of_the_equilibrium_profile():
    """The equipartition measure on the continuum equilibrium profile of a
    flat two-phase interface, phi = tanh(x / (sqrt 2 eta)) with lambda =
    (9/2)(eta^2 / beta^2) sigma^2 and beta^2 = 3 sqrt 2 sigma eta (eq:N14,
    eq:N36): int lambda phi'^2 dx = lambda 2 sqrt 2 / (3 eta) = sigma.
    Equal densities (phi = 2 c - 1).  The central differences leave a
    relative error that falls as 1 / W^2 (-0.41% at W = 16)."""
    from physics_util import line_tension
    sigma = 1e-3
    err = {}
    for Wd in (16.0, 32.0):
        eta = Wd / (2 * np.sqrt(2))
        beta2 = 3 * np.sqrt(2) * sigma * eta
        lam = np.array([[4.5 * eta ** 2 / beta2 * sigma ** 2]])
        x = np.arange(-400, 401, dtype=float)
        c1 = 0.5 + 0.5 * np.tanh(2 * x / Wd)
        err[Wd] = line_tension(np.stack([c1, 1 - c1]), (1.0, 1.0), lam) / sigma - 1
    assert abs(err[16.0]) < 6e-3
    assert err[32.0] / err[16.0] == pytest.approx(0.25, rel=0.05)
