"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against a statement that is independent of the
oracle's own code: a value the paper prints, a closed form derived by hand, an
identity the paper states (eq:a1a/a1b), a Fourier symbol, an invariant, or a
second independent transcription (oracle.literal) on tiny grids.
"""
import numpy as np
import pytest

import workloads as W
from oracle import OracleSim
from oracle.accept import oracle_accepts
from oracle.literal import LiteralSim

CS2 = 1.0 / 3.0
CK = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]], float)


def sim(N=3, nx=8, ny=8, rho=None, sigma=1e-3, **kw):
    rho = np.ones(N) if rho is None else np.asarray(rho, float)
    sig = W.uniform_sigma(N, sigma) if np.isscalar(sigma) else sigma
    return OracleSim(N, nx, ny, sig, rho, kw.pop("mu", 0.1 * rho), **kw)


def phi_from_c(c, rho):
    """eq:N12 inverted with rho_k = rho~_k c_k (eq:N2)."""
    N = len(rho)
    a = 0.5 * (rho[:-1] + rho[-1])
    b = 0.5 * (rho[:-1] - rho[-1])
    return (rho[:-1] * c[:-1] - rho[-1] * c[-1] - b) / a


# ----------------------------------------------------------------- closure
@pytest.mark.parametrize("N", [2, 3, 4, 5, 6])
def test_closure_inverts_eq_N12_and_sums_to_one(N):
    rng = np.random.default_rng(N)
    rho = rng.uniform(0.5, 20.0, N)
    s = sim(N, rho=rho)
    for _ in range(20):
        c = rng.dirichlet(np.ones(N))
        c2, r = s.closure(phi_from_c(c, rho))
        assert np.allclose(c2, c, atol=2e-15)
        # eq:N2: rho = sum_k rho_k = sum_k rho~_k c_k
        assert r == pytest.approx(np.dot(rho, c), rel=1e-14)
        # any phi (also unphysical): the fractions sum to one (eq:N2)
        cc, _ = s.closure(rng.uniform(-3, 3, N - 1))
        assert abs(cc.sum() - 1.0) < 1e-14


def test_closure_two_phase_equal_density():
    s = sim(2)
    for phi in np.linspace(-1, 1, 11):
        c, r = s.closure([phi])
        assert c[0] == pytest.approx((1 + phi) / 2, abs=1e-16)
        assert r == pytest.approx(1.0, abs=1e-15)


# ----------------------------------------------------------- setup / lambda
@pytest.mark.parametrize("N", [3, 4, 5])
def test_L_vectors_are_half_the_order_parameter_jump(N):
    rng = np.random.default_rng(10 + N)
    rho = rng.uniform(1, 10, N)
    s = sim(N, rho=rho)
    for k in range(1, N + 1):
        for l in range(k + 1, N + 1):
            ck = np.eye(N)[k - 1]
            cl = np.eye(N)[l - 1]
            jump = phi_from_c(ck, rho) - phi_from_c(cl, rho)
            assert np.allclose(2 * s.Lvec(k, l), jump, atol=1e-15)


def test_beta_matches_paper_example():
    # Sec. 4.1: sigma = 0.01 and eta = sqrt(2) give beta = sqrt(0.06)
    s = sim(3, sigma=0.01, W=2 * np.sqrt(2) * np.sqrt(2))
    lam, b2, K, eta = s.lam()
    assert eta == pytest.approx(np.sqrt(2), rel=1e-15)
    assert b2 == pytest.approx(0.06, rel=1e-14)


def test_lambda_closed_forms():
    # N = 3, equal densities and tensions: by hand from eq:N14-N16,
    # lambda = s [[4/3, -2/3], [-2/3, 4/3]], s = (9/2) (eta^2 / beta^2) sigma^2
    s3 = sim(3, sigma=1e-3, W=4.0)
    lam, b2, K, eta = s3.lam()
    sfac = 4.5 * eta ** 2 / b2 * 1e-6
    assert np.allclose(lam, sfac * np.array([[4 / 3, -2 / 3], [-2 / 3, 4 / 3]]), rtol=1e-13)
    # values of the static-droplet configuration: lambda_11 = 2e-3,
    # lambda_12 = -1e-3, beta^2 = 6e-3, K = 3e-3
    assert lam[0, 0] == pytest.approx(2e-3, rel=1e-13)
    assert lam[0, 1] == pytest.approx(-1e-3, rel=1e-13)
    assert b2 == pytest.approx(6e-3, rel=1e-14)
    assert K == pytest.approx(3e-3, rel=1e-14)
    # N = 2: a single coefficient lambda = s
    s2 = sim(2, sigma=1e-3)
    lam2, b2, K, eta = s2.lam()
    assert lam2[0, 0] == pytest.approx(4.5 * eta ** 2 / b2 * 1e-6, rel=1e-14)


def test_non_spd_sigma_rejected():
    # one tension far above the others (violates the triangle condition)
    sig = np.array([[0, 1e-3, 1e-3], [1e-3, 0, 5e-3], [1e-3, 5e-3, 0]])
    assert not oracle_accepts(sig, np.ones(3))


# --------------------------------------------------------------- h_i, C_i
@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_h_is_derivative_of_half_bulk_energy(N):
    """eq:N17 is d/dphi_i of (1/2) sum_k c_k^2 (1 - c_k)^2 (the reading of
    the factor 2 between eq:N11 and eq:N17), checked by central differences
    of the bulk energy through the closure."""
    rng = np.random.default_rng(20 + N)
    rho = rng.uniform(1, 5, N)
    s = sim(N, rho=rho)

    def energy(phi):
        c, _ = s.closure(phi)
        return 0.5 * np.sum(c ** 2 * (1 - c) ** 2)

    for _ in range(5):
        phi = phi_from_c(rng.dirichlet(np.ones(N)), rho)
        h = s.hbulk(phi)
        eps = 1e-6
        for i in range(N - 1):
            e = np.zeros(N - 1)
            e[i] = eps
            fd = (energy(phi + e) - energy(phi - e)) / (2 * eps)
            assert h[i] == pytest.approx(fd, rel=1e-7, abs=1e-12)


# ---------------------------------------------------------------- stencils
def test_stencils_exact_on_quadratics():
    s = sim(2, nx=40, ny=40, wall_y=False)
    y, x = np.mgrid[0:40, 0:40].astype(float)
    a, b, c, d, e = 0.3, -0.7, 1.1, 0.2, -0.4
    f = a * x * x + b * x * y + c * y * y + d * x + e * y
    lap, g = s.stencils(f)
    inner = (slice(2, -2), slice(2, -2))  # away from the periodic seam
    assert np.allclose(lap[inner], 2 * a + 2 * c, atol=1e-10)
    assert np.allclose(g[0][inner], (2 * a * x + b * y + d)[inner], atol=1e-10)
    assert np.allclose(g[1][inner], (b * x + 2 * c * y + e)[inner], atol=1e-10)


@pytest.mark.parametrize("m,n", [(1, 0), (2, 3), (5, 1)])
def test_stencil_fourier_symbols(m, n):
    """Symbols of eq:N31 on D2Q9 (derived): Laplacian
    [8 (cos kx + cos ky) + 4 cos kx cos ky - 20] / 6, d/dx i sin kx (2 + cos ky) / 3."""
    nx = ny = 32
    s = sim(2, nx=nx, ny=ny)
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    kx, ky = 2 * np.pi * m / nx, 2 * np.pi * n / ny
    f = np.cos(kx * x + ky * y)
    lap, g = s.stencils(f)
    sym = (8 * (np.cos(kx) + np.cos(ky)) + 4 * np.cos(kx) * np.cos(ky) - 20) / 6
    assert np.allclose(lap, sym * f, atol=1e-13)
    dsx = np.sin(kx) * (2 + np.cos(ky)) / 3
    dsy = np.sin(ky) * (2 + np.cos(kx)) / 3
    assert np.allclose(g[0], -dsx * np.sin(kx * x + ky * y), atol=1e-13)
    assert np.allclose(g[1], -dsy * np.sin(kx * x + ky * y), atol=1e-13)


def test_wall_ghosts_are_mirrors():
    s = sim(2, nx=6, ny=6, wall_y=True)
    rng = np.random.default_rng(3)
    f = rng.normal(size=(6, 6))
    lap, g = s.stencils(f)
    # row 0 with zeta(x,-1) = zeta(x,0)
    fp = np.vstack([f[:1], f, f[-1:]])
    x = 2
    e, w = fp[1, 3], fp[1, 1]
    n, sth = fp[2, 2], fp[0, 2]
    ne, nw, se, sw = fp[2, 3], fp[2, 1], fp[0, 3], fp[0, 1]
    assert lap[0, x] == pytest.approx((4 * (e + w + n + sth) + ne + nw + se + sw - 20 * fp[1, 2]) / 6,
                                      abs=1e-13)
    assert g[1, 0, x] == pytest.approx((4 * (n - sth) + ne + nw - se - sw) / 12, abs=1e-13)


def test_mixed_gradient_exact_on_quadratics():
    """eq:N40 (two-hop term negative): per direction c the four-point
    difference is exact to second order along c, and the D2Q9 weights turn
    sum_k w_k c_k (c_k . grad f) / c_s^2 into grad f, so the stencil is exact
    on quadratics; the Laplacian stays eq:N31b."""
    s = sim(2, nx=40, ny=40, wall_y=False, grad_scheme=1)
    y, x = np.mgrid[0:40, 0:40].astype(float)
    a, b, c, d, e = 0.3, -0.7, 1.1, 0.2, -0.4
    f = a * x * x + b * x * y + c * y * y + d * x + e * y
    lap, g = s.stencils(f)
    inner = (slice(3, -3), slice(3, -3))
    assert np.allclose(lap[inner], 2 * a + 2 * c, atol=1e-10)
    assert np.allclose(g[0][inner], (2 * a * x + b * y + d)[inner], atol=1e-10)
    assert np.allclose(g[1][inner], (b * x + 2 * c * y + e)[inner], atol=1e-10)


@pytest.mark.parametrize("m,n", [(1, 0), (2, 3), (5, 1), (7, 6)])
def test_mixed_gradient_fourier_symbol(m, n):
    """Symbol of eq:N40 on D2Q9 (derived by summing the eight directions of
    exp(i k.x)): d/dx -> i [sin kx (1 + cos ky / 2) - sin 2kx (1 + cos 2ky / 2) / 6],
    purely imaginary (the biased per-direction parts cancel in pairs)."""
    nx = ny = 32
    s = sim(2, nx=nx, ny=ny, grad_scheme=1)
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    kx, ky = 2 * np.pi * m / nx, 2 * np.pi * n / ny
    f = np.cos(kx * x + ky * y)
    _, g = s.stencils(f)
    sx = np.sin(kx) * (1 + np.cos(ky) / 2) - np.sin(2 * kx) * (1 + np.cos(2 * ky) / 2) / 6
    sy = np.sin(ky) * (1 + np.cos(kx) / 2) - np.sin(2 * ky) * (1 + np.cos(2 * kx) / 2) / 6
    assert np.allclose(g[0], -sx * np.sin(kx * x + ky * y), atol=1e-13)
    assert np.allclose(g[1], -sy * np.sin(kx * x + ky * y), atol=1e-13)


def test_mixed_gradient_wall_ghosts_two_deep():
    """Next to a wall the two-hop stencil reads mirror ghosts two rows deep:
    zeta(x, -1) = zeta(x, 0), zeta(x, -2) = zeta(x, 1)."""
    s = sim(2, nx=7, ny=6, wall_y=True, grad_scheme=1)
    rng = np.random.default_rng(4)
    f = rng.normal(size=(6, 7))
    _, g = s.stencils(f)
    fp = np.vstack([f[1::-1], f, f[:-3:-1]])   # two mirrored ghost rows each side

    def z(x, y):
        return fp[y + 2, x % 7]

    for y in (0, 1, 5):
        x = 3
        gy = (24 * (z(x, y + 1) - z(x, y - 1)) - 4 * (z(x, y + 2) - z(x, y - 2)) +
              6 * ((z(x + 1, y + 1) + z(x - 1, y + 1)) - (z(x + 1, y - 1) + z(x - 1, y - 1))) -
              ((z(x + 2, y + 2) + z(x - 2, y + 2)) - (z(x + 2, y - 2) + z(x - 2, y - 2)))) / 48
        assert g[1, y, x] == pytest.approx(gy, abs=1e-13)


# ------------------------------------------------------ moment identities
def test_geq_and_force_moments_eq_a1():
    """Moment conditions eq:a1a / eq:a1b (appendix)."""
    rng = np.random.default_rng(5)
    s = sim(3, rho0=0.7)
    for _ in range(10):
        rho, p = rng.uniform(0.5, 3), rng.normal() * 1e-3
        u, F, gr, J = (rng.normal(size=2) * 1e-2 for _ in range(4))
        tg = rng.uniform(0.6, 2.0)
        geq, G = s.node_dists(rho, p, u, F, gr, J, tg)
        assert geq.sum() == pytest.approx(0.7, abs=1e-15)
        assert np.allclose(CK.T @ geq, rho * u, atol=1e-16)
        M2 = np.einsum("ka,kb,k->ab", CK, CK, geq)
        assert np.allclose(M2, p * np.eye(2) + rho * np.outer(u, u), atol=1e-16)
        M3 = np.einsum("ka,kb,kc,k->abc", CK, CK, CK, geq)
        D = np.zeros((2, 2, 2))
        for a in range(2):
            for b in range(2):
                for c in range(2):
                    D[a, b, c] = rho * CS2 * ((a == b) * u[c] + (a == c) * u[b] + (b == c) * u[a])
        assert np.allclose(M3, D, atol=1e-16)
        assert G.sum() == pytest.approx(u @ gr, abs=1e-17)
        assert np.allclose(CK.T @ G, F, atol=1e-17)
        G2 = np.einsum("ka,kb,k->ab", CK, CK, G)
        Jt = np.outer(J, u) / (tg - 0.5)
        exp = (np.outer(u, F) + np.outer(F, u) + CS2 * (np.outer(u, gr) + np.outer(gr, u))
               + CS2 * (u @ gr) * np.eye(2) + 0.5 * (Jt + Jt.T))
        assert np.allclose(G2, exp, atol=1e-17)


def test_ch_equilibrium_moments():
    """h^eq of eq:N25 carries phi, phi u and c_s^2 eta_i C_i I as its zeroth,
    first and second moments (what the Chapman-Enskog recovery of eq:N19c
    with m_i = eta_i c_s^2 (tau_i - 1/2), eq:N30, rests on)."""
    rng = np.random.default_rng(6)
    s = sim(3, mobility=[0.1, 0.05], tau_phi=[0.8, 1.1])
    for i, (m, t) in enumerate([(0.1, 0.8), (0.05, 1.1)], start=1):
        eta_i = m / (CS2 * (t - 0.5))
        phi, C = rng.uniform(-1, 1), rng.normal() * 1e-3
        u = rng.normal(size=2) * 1e-2
        h = s.node_heq(i, phi, C, u)
        assert h.sum() == pytest.approx(phi, abs=1e-16)
        assert np.allclose(CK.T @ h, phi * u, atol=1e-17)
        assert np.allclose(np.einsum("ka,kb,k->ab", CK, CK, h), CS2 * eta_i * C * np.eye(2),
                           atol=1e-17)


# --------------------------------------------------------- whole-step pins
@pytest.mark.parametrize("N,wall", [(3, False), (4, True), (5, False), (5, True)])
def test_mass_conservation_and_partition_of_unity(N, wall):
    w = W.random_smooth(N, 24, 20, seed=40 + N, wall_y=wall, accept=oracle_accepts)
    s = OracleSim(**w.params())
    s.init(w.c, w.u)
    m0 = s.mass()
    s.step(300)
    c, u, p = s.macro()
    assert np.all(np.abs(s.mass() - m0) <= 1e-12 * np.abs(m0).max())
    assert np.max(np.abs(c.sum(axis=0) - 1.0)) < 1e-14
    assert np.all(np.isfinite(u)) and np.all(np.isfinite(p))


def test_uniform_mixture_stays_uniform():
    """A spatially uniform mixture at rest has no gradients, so no force and
    no flux: every node evolves identically (bitwise) and the state stays
    the initial one up to round-off (phi is re-summed every step)."""
    N = 3
    c = np.stack([np.full((8, 10), v) for v in (0.2, 0.5, 0.3)])
    s = OracleSim(N, 10, 8, W.uniform_sigma(3, 1e-3), np.array([1.0, 2.0, 3.0]),
                  np.array([0.1, 0.2, 0.3]))
    s.init(c)
    h0, g0, _, _ = s.get_state()
    s.step(25)
    h1, g1, _, _ = s.get_state()
    assert np.all(h1 == h1[..., :1, :1]) and np.all(g1 == g1[..., :1, :1])
    assert np.max(np.abs(h1 - h0)) < 1e-14 and np.array_equal(g0, g1)
    cc, u, p = s.macro()
    assert np.all(u == 0.0) and np.all(p == 0.0)
    assert np.max(np.abs(cc - c)) < 1e-14


def test_rho0_does_not_change_results():
    w = W.random_smooth(3, 16, 12, seed=9, accept=oracle_accepts)
    out = []
    for r0 in (1.0, 0.0):
        s = OracleSim(**w.params(), rho0=r0)
        s.init(w.c, w.u)
        s.step(40)
        out.append(s.macro())
    for a, b in zip(*out):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("N", [2, 3, 4, 5])
@pytest.mark.parametrize("wall", [False, True])
@pytest.mark.parametrize("shape", [(8, 8), (12, 10)])
@pytest.mark.parametrize("grad_scheme", [0, 1])
def test_c_oracle_matches_literal_transcription(N, wall, shape, grad_scheme):
    nx, ny = shape
    w = W.random_smooth(N, nx, ny, seed=60 + N + nx, wall_y=wall, accept=oracle_accepts)
    w.grad_scheme = grad_scheme
    a = OracleSim(**w.params())
    b = LiteralSim(**w.params())
    a.init(w.c, w.u)
    b.init(w.c, w.u)
    a.step(50)
    b.step(50)
    for x, y in zip(a.macro(), b.macro()):
        assert np.max(np.abs(x - y)) < 1e-13


# --------------------------------------------------------- physics pins
def test_taylor_green_viscous_decay():
    """Single-phase limit (c_1 = 1 everywhere: F, grad rho, J~ vanish): the
    shear-wave amplitude decays as exp(-2 nu k^2 t), nu = c_s^2 (tau_g - 1/2)
    (eq:N21_1)."""
    n, nu = 64, 0.1
    w = W.taylor_green(n, amp=1e-3, nu=nu)
    s = OracleSim(**w.params())
    s.init(w.c, w.u)
    k = 2 * np.pi / n
    y, x = np.mgrid[0:n, 0:n].astype(float)
    shape = np.sin(k * x) * np.cos(k * y)

    def amp():
        _, u, _ = s.macro()
        return np.sum(u[1] * shape) / np.sum(shape * shape)

    s.step(100)
    a1 = amp()
    s.step(400)
    a2 = amp()
    rate = -np.log(a2 / a1) / 400
    assert rate == pytest.approx(2 * nu * k * k, rel=0.01)


def test_cahn_hilliard_linear_dispersion():
    """N = 2, equal densities, small cosine perturbation of a near-pure phase:
    linearising eq:N19c with C of eq:N18 gives the decay rate
    m k^2 (lambda k_d^2 + K h'(phi_0)), with k_d^2 the symbol of eq:N31b and
    h' = (1 - 6 c_0 + 6 c_0^2) / 2 (from eq:N17, derived)."""
    n, c0, m = 64, 0.05, 1.0
    w = W.cosine_perturbation(n, c0=c0, amp=1e-5, mobility=m, sigma=1e-2)
    s = OracleSim(**w.params())
    lam, b2, K, eta = s.lam()
    s.init(w.c, w.u)
    k = 2 * np.pi / n
    x = np.arange(n)
    mode = np.cos(k * x)

    def amp():
        c, _, _ = s.macro()
        return np.mean(c[1], axis=0) @ mode / (mode @ mode)

    s.step(200)
    a1 = amp()
    s.step(2000)
    a2 = amp()
    rate = -np.log(a2 / a1) / 2000
    kd2 = -(8 * (np.cos(k) + 1) + 4 * np.cos(k) - 20) / 6
    hp = (1 - 6 * c0 + 6 * c0 * c0) / 2
    theory = m * k * k * (lam[0, 0] * kd2 + K * hp)
    assert rate == pytest.approx(theory, rel=0.02)
