"""Transport pins of the FP64 oracle: the two pieces that no static or
single-phase pin reaches.

1. The Cahn-Hilliard source term R_k (eq:N26) with the backward-Euler time
   derivative of phi_i u (eq:N27).  Pin: in a periodic box of equal-density
   fluid pushed by a uniform body force, every parcel is accelerated alike,
   so a band of one phase is carried with the fluid (Galilean consistency of
   the advective flux phi u in eq:N13).  The fluid's displacement after T
   steps is fixed in closed form by eq:N22_1: the momentum before collision
   at step t is rho g t, after collision rho g (t + 1), and streaming moves
   mass by the post-collision momentum, so the fluid moves by
   g T (T + 1) / 2.  The band's centre of mass must move by the same amount.
   Summing eq:N24 over the domain shows what each reading predicts: the
   first moments of h^eq (eq:N25) and R_k are phi u and (1 - 1/(2 tau))
   d_t(phi u), the collision keeps a fraction (1 - 1/tau) of the rest and
   streaming conserves it, which leaves only a start-up term of
   (g/2)(tau - 1/2)(1 - (1 - 1/tau)^T) because the stored initial u (0)
   differs from the first computed u (g/2).  With the sign of R_k flipped,
   R_k dropped, or d_t(phi u) formed with one velocity for both times
   (phi u_prev - phi_prev u_prev or phi u - phi_prev u), the band lags the
   fluid by 0.3 to 0.6 g per step; those planted variants (test side, on the
   NumPy transcription) must fail.

2. The per-node NS relaxation time tau_g = 1/2 + mu / (rho c_s^2) with
   mu = sum_k mu~_k c_k (eq:N21_1 with the viscosity of Sec. 2).  Pin:
   steady body-force-driven flow between halfway bounce-back walls across
   two flat interfaces (a band of phase 1 centred in the channel, phase 2
   next to both walls) with mu~_k / rho~_k different in the two phases.  The
   steady momentum balance of the unidirectional flow is
   d/dy (mu du/dy) = -rho g; by symmetry the shear stress vanishes at the
   centre line, so mu(y) u'(y) = -g int_centre^y rho, and the velocity rise
   from a node near the wall to the centre line is the quadrature of that
   stress over mu (Poiseuille flow in layers, a textbook closed form evaluated
   on the measured c profile).  A constant tau_g, the kinematic viscosity
   interpolated instead of the dynamic one, a harmonic mean, or the c_s^2
   dropped, all planted on the test side, miss it by 10% to 200%.
"""
import numpy as np
import pytest

import workloads as W
from oracle import OracleSim
from oracle.literal import LiteralSim

CS2 = 1.0 / 3.0


# ---------------------------------------------------------------- planted
class FlippedSource(LiteralSim):
    """PLANTED MISTAKE: R_k with the opposite sign."""

    def flux_rate(self, phi, u):
        return -super().flux_rate(phi, u)


class NoSource(LiteralSim):
    """PLANTED MISTAKE: R_k left out."""

    def flux_rate(self, phi, u):
        return 0.0 * super().flux_rate(phi, u)


class PreviousVelocityOnly(LiteralSim):
    """PLANTED MISTAKE: d_t(phi u) formed with the previous u at both times."""

    def flux_rate(self, phi, u):
        return (phi - self.pphi)[:, None] * self.pu[None]


class CurrentVelocityOnly(LiteralSim):
    """PLANTED MISTAKE: d_t(phi u) formed with the current u at both times."""

    def flux_rate(self, phi, u):
        return (phi - self.pphi)[:, None] * u[None]


class ConstantTau(LiteralSim):
    """PLANTED MISTAKE: tau_g of phase 1 everywhere."""

    def tau_g(self, c, rho):
        return 0.5 + self.mt[0] / (self.rt[0] * CS2) + 0.0 * rho


class KinematicMean(LiteralSim):
    """PLANTED MISTAKE: nu = sum_k (mu~_k / rho~_k) c_k instead of mu / rho."""

    def tau_g(self, c, rho):
        return 0.5 + np.einsum("k,kyx->yx", self.mt / self.rt, c) / CS2


class HarmonicMean(LiteralSim):
    """PLANTED MISTAKE: harmonic mean of the dynamic viscosities."""

    def tau_g(self, c, rho):
        mu = 1.0 / np.einsum("k,kyx->yx", 1.0 / self.mt, c)
        return 0.5 + mu / (rho * CS2)


class NoSoundSpeed(LiteralSim):
    """PLANTED MISTAKE: tau_g = 1/2 + mu / rho (c_s^2 dropped)."""

    def tau_g(self, c, rho):
        return 0.5 + np.einsum("k,kyx->yx", self.mt, c) / rho


# ------------------------------------------------- 1. source term R_k
NXB, NYB = 256, 4
G_ACC, T_ACC = 8e-5, 500


def _bands(N, W0):
    x = np.arange(NXB)[None, :] * np.ones((NYB, 1))

    def band(a, b):
        return 0.5 * (np.tanh(2 * (x - a) / W0) - np.tanh(2 * (x - b) / W0))

    c1 = band(50, 106)
    if N == 2:
        return np.stack([c1, 1 - c1]), x
    c3 = band(140, 180)
    return np.stack([c1, 1 - c1 - c3, c3]), x


def _band_shift(cls, N, tau, T=T_ACC):
    """Displacement of the phase-1 band's centre of mass after T steps of
    uniform acceleration G_ACC along x (equal densities, W = 8)."""
    c, x = _bands(N, 8.0)
    rho = np.ones(N)
    s = cls(N, NXB, NYB, W.uniform_sigma(N, 1e-3), rho, 0.1 * rho, W=8.0, gx=G_ACC,
            tau_phi=tau)
    s.init(c, None)
    s.step(T)
    c1 = s.macro()[0][0]
    cen = lambda f: float((f * x).sum() / f.sum())
    return cen(c1) - cen(c[0])


def _fluid_shift(tau, T=T_ACC):
    """Closed form: fluid displacement g T (T+1)/2 plus the start-up term."""
    g = G_ACC
    return g * T * (T + 1) / 2 - 0.5 * g * (tau - 0.5) * (1 - (1 - 1 / tau) ** T)


@pytest.mark.parametrize("N", [2, 3])
@pytest.mark.parametrize("tau", [0.8, 1.3])
def test_phase_band_moves_with_the_accelerated_fluid(N, tau):
    d = _band_shift(OracleSim, N, tau)
    exp = _fluid_shift(tau)
    assert abs(exp - 10.02) < 1e-3          # 10 lattice spacings
    # the wrong readings miss by >= 0.3 g per step (150 g here); measured:
    # within 0.2 g at tau = 0.8 and 6.4 g at tau = 1.3 (discretisation of
    # the W = 8 profile)
    assert abs(d - exp) < 0.02 * G_ACC * T_ACC, (d, exp)


@pytest.mark.parametrize("cls", [FlippedSource, NoSource, PreviousVelocityOnly,
                                 CurrentVelocityOnly])
def test_band_pin_rejects_planted_source_terms(cls):
    # the transcription itself passes ...
    assert abs(_band_shift(LiteralSim, 2, 0.8, T=200) - _fluid_shift(0.8, T=200)) < 2 * G_ACC
    # ... the planted variants lag by >= 0.3 g per step
    d = _band_shift(cls, 2, 0.8, T=200)
    assert abs(d - _fluid_shift(0.8, T=200)) > 40 * G_ACC


# --------------------------------------------- 2. per-node tau_g
NXP, NYP, HW = 4, 32, 8
RHO_P = np.array([1.0, 3.0])
MU_P = np.array([0.1, 0.9])   # nu = 0.1 and 0.3: tau_g 0.8 and 1.4
G_P = 1e-6


def _channel():
    y = np.arange(NYP)[:, None] * np.ones((1, NXP))
    yc = (NYP - 1) / 2
    c1 = 0.5 * (np.tanh(2 * (y - (yc - HW)) / 4.0) - np.tanh(2 * (y - (yc + HW)) / 4.0))
    return np.stack([c1, 1 - c1])


def _rise_error(c, u):
    """Relative error of the velocity rise from node 2 to the centre line
    against the quadrature of the layered-Poiseuille stress over mu."""
    mu = (MU_P[:, None] * c[:, :, 0]).sum(0)
    rho = (RHO_P[:, None] * c[:, :, 0]).sum(0)
    cum = np.cumsum(rho)
    stress = -G_P * (cum - cum[-1] / 2)[:-1]      # at the half-nodes j + 1/2
    mu_h = 0.5 * (mu[1:] + mu[:-1])
    j0, jc = 2, NYP // 2 - 1
    pred = np.sum(stress[j0:jc] / mu_h[j0:jc])
    ux = u[0][:, 0]
    return (ux[jc] - ux[j0]) / pred - 1.0


def _channel_sim(cls):
    return cls(2, NXP, NYP, W.uniform_sigma(2, 1e-3), RHO_P, MU_P, W=4.0, gx=G_P, wall_y=True)


@pytest.fixture(scope="module")
def steady_channel():
    s = _channel_sim(OracleSim)
    s.init(_channel(), None)
    s.step(8000)
    return s


def test_layered_poiseuille_follows_the_local_viscosity(steady_channel):
    s = steady_channel
    c, u, _ = s.macro()
    f = s.fields()
    # tau_g really varies: 0.8 in phase 1 at the centre, 1.4 next to the walls
    assert f["taug"][NYP // 2, 0] == pytest.approx(0.8, abs=1e-3)
    assert f["taug"][0, 0] == pytest.approx(1.4, abs=1e-3)
    e0 = _rise_error(c, u)
    s.step(1000)
    c, u, _ = s.macro()
    e1 = _rise_error(c, u)
    assert abs(e1 - e0) < 1e-4               # steady
    assert abs(e1) < 0.03, e1                # measured -0.95% (W = 4; -0.31% at W = 8)


@pytest.mark.parametrize("cls", [ConstantTau, KinematicMean, HarmonicMean, NoSoundSpeed])
def test_poiseuille_pin_rejects_planted_viscosities(steady_channel, cls):
    # start from the converged oracle state; the planted relaxation time then
    # moves the profile towards its own steady state (time constant ~1000 steps)
    h, g, pp, pu = steady_channel.get_state()
    s = _channel_sim(cls)
    s.init(_channel(), None)
    s.h, s.g, s.pphi, s.pu = h.copy(), g.copy(), pp.copy(), pu.copy()
    s.step(2500)
    c, u, _ = s.macro()
    assert abs(_rise_error(c, u)) > 0.06
