"""Pins of the oracle's second total-force distribution (Remark 1, Sec. 3.1):
G_k without the J~ u / (tau_g - 1/2) tensor term and F = -div(J~ u) + F_s + G,
component a of the divergence being sum_b d_b (J~_b u_a) (the identity
J~ . grad u = div(J~ u) - (div J~) u of Sec. 2 fixes the index order).

The planted mistake lives here, on the test side: ``SwappedDivergence`` is
the NumPy transcription with the divergence taken over the other index,
sum_b d_b (J~_a u_b).  The tests below must tell it apart from form 1; the
oracle itself accepts force_form 0 and 1 only.
"""
import numpy as np
import pytest

import workloads as W
from oracle import OracleSim
from oracle.accept import oracle_accepts
from oracle.literal import LiteralSim

CS2 = 1.0 / 3.0


class SwappedDivergence(LiteralSim):
    """PLANTED MISTAKE (tests only): Remark 1's divergence over the wrong index."""

    def flux_divergence(self, J, u):
        return np.stack([sum(self.grad(J[a] * u[b])[b] for b in range(2)) for a in range(2)])


CK = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]], float)


def test_remark1_force_moments():
    """Moments of the Remark 1 distribution: sum G = u.grad rho, sum c G = F,
    sum c c G = uF + Fu + cs^2 (u grad rho + grad rho u) + cs^2 (u.grad rho) I
    (eq:a1b without the J~ term); J~ must not enter at all."""
    rng = np.random.default_rng(8)
    s = OracleSim(3, 8, 8, W.uniform_sigma(3, 1e-3), np.array([1.0, 2.0, 3.0]),
                  np.array([0.1, 0.2, 0.3]), force_form=1)
    for _ in range(10):
        rho, p = rng.uniform(0.5, 3), rng.normal() * 1e-3
        u, F, gr, J = (rng.normal(size=2) * 1e-2 for _ in range(4))
        tg = rng.uniform(0.6, 2.0)
        _, G = s.node_dists(rho, p, u, F, gr, J, tg)
        _, G0 = s.node_dists(rho, p, u, F, gr, np.zeros(2), tg)
        assert np.array_equal(G, G0)
        assert G.sum() == pytest.approx(u @ gr, abs=1e-17)
        assert np.allclose(CK.T @ G, F, atol=1e-17)
        G2 = np.einsum("ka,kb,k->ab", CK, CK, G)
        exp = (np.outer(u, F) + np.outer(F, u) + CS2 * (np.outer(u, gr) + np.outer(gr, u))
               + CS2 * (u @ gr) * np.eye(2))
        assert np.allclose(G2, exp, atol=1e-17)


@pytest.mark.parametrize("wall", [False, True])
def test_forms_identical_when_flux_vanishes(wall):
    """Equal densities make kappa_i = 1 - N gamma_i / Gamma zero, so J~ = 0
    (eq:N18) and both force distributions are the same arithmetic."""
    w = W.random_smooth(4, 12, 10, seed=71, wall_y=wall, accept=oracle_accepts, unequal=False)
    runs = []
    for ff in (0, 1):
        s = OracleSim(**w.params(), force_form=ff)
        s.init(w.c, w.u)
        s.step(40)
        runs.append(s.macro())
    for a, b in zip(*runs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("wall", [False, True])
@pytest.mark.parametrize("planted", [False, True])
def test_divergence_of_flux_times_uniform_velocity(wall, planted):
    """With the previous velocity uniform (u = U at t = 0), div(J~ U) is U
    times div J~ by linearity of the stencil: F(form 1) - F(eq:N20_1 form) =
    -U (div J~), with div J~ from the oracle's eq:N31a stencil applied to the
    J~ field.  The planted form gives (U . grad) J~ instead and must fail."""
    nx, ny = 24, 16
    w = W.random_smooth(3, nx, ny, seed=72, wall_y=wall, accept=oracle_accepts)
    U = np.array([0.013, -0.021])
    u = np.broadcast_to(U[:, None, None], (2, ny, nx)).copy()
    s0 = OracleSim(**w.params(), force_form=0)
    s0.init(w.c, u)
    f0 = s0.fields()
    if planted:
        s1 = SwappedDivergence(**w.params(), force_form=1)
        s1.init(w.c, u)
        F1 = s1.macro_all()["F"]
    else:
        s1 = OracleSim(**w.params(), force_form=1)
        s1.init(w.c, u)
        F1 = s1.fields()["F"]
    J = f0["J"]
    _, gJx = s0.stencils(J[0])
    _, gJy = s0.stencils(J[1])
    divJ = gJx[0] + gJy[1]
    exp = -U[:, None, None] * divJ[None]
    got = F1 - f0["F"]
    assert np.max(np.abs(divJ)) > 1e-7
    err = np.max(np.abs(got - exp)) / np.max(np.abs(exp))
    if planted:
        assert err > 0.1
    else:
        assert err < 1e-9


@pytest.mark.parametrize("N", [2, 3, 5])
@pytest.mark.parametrize("wall", [False, True])
@pytest.mark.parametrize("grad_scheme", [0, 1])
def test_remark1_c_oracle_matches_literal_transcription(N, wall, grad_scheme):
    w = W.random_smooth(N, 12, 10, seed=80 + N, wall_y=wall, accept=oracle_accepts)
    w.grad_scheme = grad_scheme
    a = OracleSim(**w.params(), force_form=1)
    b = LiteralSim(**w.params(), force_form=1)
    a.init(w.c, w.u)
    b.init(w.c, w.u)
    a.step(50)
    b.step(50)
    for x, y in zip(a.macro(), b.macro()):
        assert np.max(np.abs(x - y)) < 1e-13


def test_eq_N20_1_carries_the_symmetric_half_of_the_flux_term():
    """Chapman-Enskog reading of the two forms.  eq:N20_1 puts J~ u into G_k
    only through its contraction with (c c - c_s^2 I), so on the lattice its
    second moment is the symmetric part of J~ u (eq:a1b prints it
    unsymmetrised) and it recovers -div of (J~ u + u J~) / 2; Remark 1
    recovers -div(J~ u).  With J~ along x and u along y, the planted form
    (indices swapped) drops the term from the y momentum, Remark 1 has all
    of it and eq:N20_1 half: the eq:N20_1 run lies midway between the other
    two.  Set-up: a relaxing (twice too wide) flat interface pair normal to
    x, density ratio 10, uniform u_y."""
    nx, ny = 64, 4
    x = np.arange(nx)[None, :] * np.ones((ny, 1))
    Wd = 4.0
    c1 = 0.5 * (np.tanh(2 * (x - 16) / (2 * Wd)) - np.tanh(2 * (x - 48) / (2 * Wd)))
    c = np.stack([c1, 1 - c1])
    u = np.zeros((2, ny, nx))
    u[1] = 0.02
    rho = np.array([10.0, 1.0])
    uy = {}
    for ff in (0, 1, 2):
        # 2 = the planted swapped-index form (test side)
        cls = SwappedDivergence if ff == 2 else OracleSim
        s = cls(2, nx, ny, W.uniform_sigma(2, 1e-3), rho, 0.1 * rho, W=Wd,
                force_form=min(ff, 1))
        s.init(c, u)
        s.step(50)
        uy[ff] = s.macro()[1][1]
    d1 = (uy[1] - uy[0]).ravel()
    d2 = (uy[2] - uy[0]).ravel()
    assert np.max(np.abs(d1)) > 1e-6
    corr = d1 @ d2 / np.sqrt((d1 @ d1) * (d2 @ d2))
    assert corr < -0.98
    assert 0.8 < np.linalg.norm(d1) / np.linalg.norm(d2) < 1.25
