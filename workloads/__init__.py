"""Seeded synthetic inputs for the N-phase phase-field LB workloads.

This module only draws and lays out inputs: initial volume fractions built
from the diffuse tanh profiles of the paper's test problems (eq:N31_a,
eq:N35, eq:N38, eq:N39), initial velocities, pairwise surface tensions,
densities and viscosities, and the serving request stream.  It holds none of
the method's arithmetic, so both the FP64 oracle and the GPU path take their
inputs from here.

Coordinates: node (x, y) sits at integer position (x, y), x fastest in
memory; arrays have shape (N, ny, nx).  The tanh argument of the paper,
(R - r) / (sqrt(2) eta), is written with the interface width W = 2 sqrt(2) eta
as 2 (R - r) / W.

Every draw takes an explicit seed derived from BASE_SEED.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Sequence

import numpy as np

BASE_SEED = 1904


def _profile(d: np.ndarray, W: float) -> np.ndarray:
    """0.5 + 0.5 tanh(2 d / W): the paper's diffuse profile at signed distance d."""
    return 0.5 + 0.5 * np.tanh(2.0 * d / W)


def grid(nx: int, ny: int):
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    return x, y


def disc(nx: int, ny: int, xc: float, yc: float, R: float, W: float) -> np.ndarray:
    """Diffuse disc of radius R centred at (xc, yc) (eq:N31_a pattern)."""
    x, y = grid(nx, ny)
    r = np.sqrt((x - xc) ** 2 + (y - yc) ** 2)
    return _profile(R - r, W)


@dataclasses.dataclass
class Workload:
    """Everything needed to create and initialise one domain."""
    name: str
    N: int
    nx: int
    ny: int
    sigma: np.ndarray           # N x N, symmetric, zero diagonal
    rho: np.ndarray             # N densities
    mu: np.ndarray              # N dynamic viscosities
    c: np.ndarray               # (N, ny, nx) initial volume fractions
    u: Optional[np.ndarray]     # (2, ny, nx) initial velocity or None
    mobility: float = 0.1
    tau_phi: float = 0.8
    W: float = 4.0
    wall_y: bool = False
    gx: float = 0.0
    gy: float = 0.0
    steps: int = 1000
    precision: int = 64
    note: str = ""
    grad_scheme: int = 0        # 0: eq:N31a central, 1: eq:N40 mixed
    nz: int = 1                 # > 1: a 3-D (D3Q15) workload, fields (.., nz, ny, nx)
    wall_z: bool = False        # 3-D: walls below plane 0 and above plane nz - 1
    gz: float = 0.0

    def params(self) -> dict:
        if self.nz > 1:
            return dict(N=self.N, nx=self.nx, ny=self.ny, nz=self.nz, sigma=self.sigma,
                        rho=self.rho, mu=self.mu, mobility=self.mobility, tau_phi=self.tau_phi,
                        W=self.W, wall_z=self.wall_z, gx=self.gx, gy=self.gy, gz=self.gz)
        return dict(N=self.N, nx=self.nx, ny=self.ny, sigma=self.sigma, rho=self.rho,
                    mu=self.mu, mobility=self.mobility, tau_phi=self.tau_phi, W=self.W,
                    wall_y=self.wall_y, gx=self.gx, gy=self.gy, grad_scheme=self.grad_scheme)


def uniform_sigma(N: int, value: float) -> np.ndarray:
    s = np.full((N, N), float(value))
    np.fill_diagonal(s, 0.0)
    return s


def draw_sigma(N: int, seed: int, lo: float = 0.5e-3, hi: float = 2e-3,
               accept: Optional[Callable[[np.ndarray, np.ndarray], bool]] = None,
               rho: Optional[np.ndarray] = None, max_draws: int = 1000):
    """Pairwise tensions sigma_kl ~ U[lo, hi], redrawn until
    ``accept(sigma, rho)`` (the caller's well-posedness check, e.g. an SPD
    mixing matrix for densities ``rho``) says yes.

    Returns (sigma, number_of_redraws)."""
    rng = np.random.default_rng(seed)
    for it in range(max_draws):
        s = np.zeros((N, N))
        iu = np.triu_indices(N, 1)
        s[iu] = rng.uniform(lo, hi, size=len(iu[0]))
        s = s + s.T
        if accept is None or accept(s, rho):
            return s, it
    raise RuntimeError("no acceptable sigma draw")


# ---------------------------------------------------------------------------
# The configurations of the workload table
# ---------------------------------------------------------------------------

def static_droplet(nx: int = 100, ny: int = 100, R: float = 25.0, W: float = 4.0,
                   sigma: float = 1e-3, precision: int = 64, steps: int = 2000,
                   tau_g: float = 1.0) -> Workload:
    """N=3 static droplet: phase-2 disc of radius R centred in phase 1,
    phase 3 absent (eq:N31_a pattern); periodic; equal densities; viscosity
    chosen so that tau_g = 1.0."""
    c2 = disc(nx, ny, nx / 2.0, ny / 2.0, R, W)
    c3 = np.zeros_like(c2)
    c1 = 1.0 - c2 - c3
    nu = (tau_g - 0.5) / 3.0
    return Workload("static_droplet_N3", 3, nx, ny, uniform_sigma(3, sigma), np.ones(3),
                    np.full(3, nu), np.stack([c1, c2, c3]), None, mobility=0.1,
                    tau_phi=0.8, W=W, steps=steps, precision=precision)


def two_phase_droplet(nx: int = 100, ny: int = 100, R: float = 25.0, W: float = 4.0,
                      sigma: float = 1e-3, mobility: float = 0.2, steps: int = 2000,
                      tau_g: float = 1.0) -> Workload:
    """The N=2 counterpart of static_droplet (phase 3 removed)."""
    c2 = disc(nx, ny, nx / 2.0, ny / 2.0, R, W)
    nu = (tau_g - 0.5) / 3.0
    return Workload("static_droplet_N2", 2, nx, ny, uniform_sigma(2, sigma), np.ones(2),
                    np.full(2, nu), np.stack([1.0 - c2, c2]), None, mobility=mobility,
                    tau_phi=0.8, W=W, steps=steps)


def liquid_lens(nx: int = 400, ny: int = 200, R: float = 40.0, W: float = 4.0,
                s12: float = 1e-3, s13: float = 1e-3, s23: float = 1e-3,
                rho=(1.0, 1.0, 1.0), tau_g: float = 0.8, mobility: float = 0.1,
                precision: int = 64, steps: int = 20000) -> Workload:
    """N=3 liquid lens (eq:N35 pattern with phase 3 as the lens): lens disc of
    radius R at the centre of a flat phase-1 / phase-2 interface, phase 2 on
    top; periodic in x, halfway bounce-back walls in y."""
    xc, yc = nx / 2.0, ny / 2.0
    c3 = disc(nx, ny, xc, yc, R, W)
    x, y = grid(nx, ny)
    c2 = np.maximum(_profile(y - yc, W) - c3, 0.0)
    c1 = 1.0 - c2 - c3
    sig = np.array([[0.0, s12, s13], [s12, 0.0, s23], [s13, s23, 0.0]])
    rho = np.asarray(rho, dtype=np.float64)
    nu = (tau_g - 0.5) / 3.0
    return Workload("liquid_lens_N3", 3, nx, ny, sig, rho, rho * nu, np.stack([c1, c2, c3]),
                    None, mobility=mobility, tau_phi=0.8, W=W, wall_y=True, steps=steps,
                    precision=precision)


def droplet_collision(side: int = 512, W: float = 4.0, seed: int = BASE_SEED + 3,
                      accept=None, precision: int = 32, steps: int = 50000,
                      speed: float = 0.01) -> Workload:
    """N=4 droplet collision: phase 1 is the matrix; phases 2, 3, 4 are discs
    of radius 48/512 * side at (144, 256), (368, 256), (256, 400) (scaled) moving
    with (+v, 0), (-v, 0), (0, -v); u = sum_d c_d v_d; periodic.  sigma_kl ~
    U[0.5e-3, 2e-3], densities rho_1 = 1, rho_2..4 ~ U[1, 3] from the same
    seed stream; mu_k = 0.1 rho_k (tau_g = 0.8)."""
    s = side / 512.0
    R = 48.0 * s
    centres = [(144 * s, 256 * s, speed, 0.0), (368 * s, 256 * s, -speed, 0.0),
               (256 * s, 400 * s, 0.0, -speed)]
    cs = [disc(side, side, xc, yc, R, W) for xc, yc, _, _ in centres]
    c1 = 1.0 - sum(cs)
    c = np.stack([c1] + cs)
    u = np.zeros((2, side, side))
    for cd, (_, _, vx, vy) in zip(cs, centres):
        u[0] += cd * vx
        u[1] += cd * vy
    rng = np.random.default_rng(seed + 1000)
    rho = np.concatenate([[1.0], rng.uniform(1.0, 3.0, size=3)])
    sigma, redraws = draw_sigma(4, seed, accept=accept, rho=rho)
    return Workload("droplet_collision_N4", 4, side, side, sigma, rho, 0.1 * rho, c, u,
                    mobility=0.1, tau_phi=0.8, W=W, steps=steps, precision=precision,
                    note=f"sigma redraws={redraws}")


def floating_puddle(nx: int = 400, ny: int = 200, R: float = 30.0, W: float = 4.0,
                    g: float = 1e-4, sigma=(0.01, 0.01, 0.01), rho=(3.0, 1.0, 6.0),
                    precision: int = 64, steps: int = 200000) -> Workload:
    """A phase-1 droplet at the flat interface between a light phase 2 (top)
    and a heavy phase 3 (bottom), eq:N35 layout, under gravity g downward
    (-y), walls in y (Sec. 4.2, second part): rho = 3 : 1 : 6, sigma_12 :
    sigma_13 : sigma_23 = 1 : 1 : 1 (0.01), tau = 0.8 (mu = 0.1 rho), m =
    0.1, W = 4.  For large g it flattens into a puddle whose thickness tends
    to eq:N37."""
    xc, yc = nx / 2.0, ny / 2.0
    c1 = disc(nx, ny, xc, yc, R, W)
    _, y = grid(nx, ny)
    c2 = np.maximum(_profile(y - yc, W) - c1, 0.0)
    c3 = 1.0 - c1 - c2
    s12, s13, s23 = sigma
    sig = np.array([[0.0, s12, s13], [s12, 0.0, s23], [s13, s23, 0.0]])
    rho = np.asarray(rho, dtype=float)
    return Workload("floating_puddle_N3", 3, nx, ny, sig, rho, 0.1 * rho,
                    np.stack([c1, c2, c3]), None, mobility=0.1, tau_phi=0.8, W=W,
                    wall_y=True, gy=-g, steps=steps, precision=precision)


def four_phase_buoyancy(nx: int = 200, ny: int = 320, D: float = 60.0, W: float = 4.0,
                        sigma13: float = 0.01, g: float = 1e-5, precision: int = 64,
                        steps: int = 30000, grad_scheme: int = 0) -> Workload:
    """N=4 droplet and bubble under gravity (Sec. 4.3, eq:N38): phase 3 above
    phase 4 (interface at y0 = ny / 2), a phase-1 droplet of diameter D at
    (160, 280) inside phase 3 and a phase-2 bubble at (160, 40) inside phase
    4 (the printed centres; x is periodic, so only their common column
    matters), scaled with the domain; rho = 6 : 1 : 3 : 2, sigma_13 varied,
    every other sigma 0.01, tau = 0.8 (mu = 0.1 rho), m = 0.1, W = 4, g
    downward (-y); walls in y, periodic in x."""
    sx, sy = nx / 200.0, ny / 320.0
    R = D / 2.0
    c1 = disc(nx, ny, (160 * sx) % nx, 280 * sy, R, W)
    c2 = disc(nx, ny, (160 * sx) % nx, 40 * sy, R, W)
    _, y = grid(nx, ny)
    c3 = _profile(y - ny / 2.0, W) * (1.0 - c1)
    c4 = 1.0 - c1 - c2 - c3
    sig = uniform_sigma(4, 0.01)
    sig[0, 2] = sig[2, 0] = sigma13
    rho = np.array([6.0, 1.0, 3.0, 2.0])
    return Workload("four_phase_buoyancy_N4", 4, nx, ny, sig, rho, 0.1 * rho,
                    np.stack([c1, c2, c3, c4]), None, mobility=0.1, tau_phi=0.8, W=W,
                    wall_y=True, gy=-g, steps=steps, precision=precision,
                    grad_scheme=grad_scheme)


def five_phase_buoyancy(nx: int = 200, ny: int = 320, R: float = 30.0, W: float = 4.0,
                        g: float = 1e-5, grad_scheme: int = 1, precision: int = 64,
                        steps: int = 20000) -> Workload:
    """N=5 droplets and interface under gravity (Sec. 4.4, eq:N39): phase 4
    above phase 5 (interface at y0 = ny / 2), droplets of phases 1 and 2 at
    (60, 280) and (140, 280) inside phase 4, a bubble of phase 3 at
    (100, 40) inside phase 5 (positions for the 200 x 320 domain, scaled
    with it); rho = 6 : 4 : 1 : 2 : 3, all sigma = 0.01, tau = 0.8 (mu =
    0.1 rho), m = 0.1, W = 4 (eta = sqrt 2), gravity g downward (-y); walls
    in y, periodic in x; the paper runs it with the mixed gradient scheme
    of eq:N40."""
    sx, sy = nx / 200.0, ny / 320.0
    c1 = disc(nx, ny, 60 * sx, 280 * sy, R, W)
    c2 = disc(nx, ny, 140 * sx, 280 * sy, R, W)
    c3 = disc(nx, ny, 100 * sx, 40 * sy, R, W)
    _, y = grid(nx, ny)
    c5 = _profile(ny / 2.0 - y, W) * (1.0 - c3)
    c4 = 1.0 - c1 - c2 - c3 - c5
    rho = np.array([6.0, 4.0, 1.0, 2.0, 3.0])
    return Workload("five_phase_buoyancy_N5", 5, nx, ny, uniform_sigma(5, 0.01), rho, 0.1 * rho,
                    np.stack([c1, c2, c3, c4, c5]), None, mobility=0.1, tau_phi=0.8, W=W,
                    wall_y=True, gy=-g, steps=steps, precision=precision,
                    grad_scheme=grad_scheme)


def bands_and_droplets(side: int = 2048, ndrop: int = 64, W: float = 4.0,
                       seed: int = BASE_SEED + 4, accept=None, precision: int = 32,
                       steps: int = 20000, rmin: float = 10.0, rmax: float = 40.0) -> Workload:
    """N=5 droplets and interfaces (eq:N39 pattern): horizontal bands of
    phases 1, 2, 3 of height side/4 stacked from y = side/8 (phase 4 fills the
    rest, across the periodic seam), plus ``ndrop`` phase-5 droplets with
    radius ~ U[rmin, rmax] at seeded, non-overlapping centres (gap >= 2W);
    the band fractions are scaled by (1 - c_5).  sigma_kl ~ U[0.5e-3, 2e-3],
    rho_k ~ U[1, 3], mu_k = 0.1 rho_k, periodic."""
    x, y = grid(side, side)
    h = side / 4.0
    y0 = side / 8.0
    bands = []
    for b in range(3):
        lo, hi = y0 + b * h, y0 + (b + 1) * h
        bands.append(0.5 * (np.tanh(2.0 * (y - lo) / W) - np.tanh(2.0 * (y - hi) / W)))
    rng = np.random.default_rng(seed)
    drops: List[tuple] = []
    tries = 0
    while len(drops) < ndrop:
        tries += 1
        if tries > 200000:
            raise RuntimeError("could not place droplets")
        r = rng.uniform(rmin, rmax)
        xc = rng.uniform(r + W, side - r - W)
        yc = rng.uniform(r + W, side - r - W)
        if all(math.hypot(xc - a, yc - b) >= r + q + 2 * W for a, b, q in drops):
            drops.append((xc, yc, r))
    c5 = np.zeros((side, side))
    for xc, yc, r in drops:
        # each droplet only touches a box around its centre
        x0, x1 = int(max(0, xc - r - 4 * W)), int(min(side, xc + r + 4 * W + 1))
        y0b, y1b = int(max(0, yc - r - 4 * W)), int(min(side, yc + r + 4 * W + 1))
        xx, yy = x[y0b:y1b, x0:x1], y[y0b:y1b, x0:x1]
        d = r - np.sqrt((xx - xc) ** 2 + (yy - yc) ** 2)
        c5[y0b:y1b, x0:x1] += _profile(d, W)
    c5 = np.minimum(c5, 1.0)
    bands = [b * (1.0 - c5) for b in bands]
    c4 = 1.0 - bands[0] - bands[1] - bands[2] - c5
    c = np.stack(bands + [c4, c5])
    rng2 = np.random.default_rng(seed + 1000)
    rho = rng2.uniform(1.0, 3.0, size=5)
    sigma, redraws = draw_sigma(5, seed + 7, accept=accept, rho=rho)
    return Workload("bands_droplets_N5", 5, side, side, sigma, rho, 0.1 * rho, c, None,
                    mobility=0.1, tau_phi=0.8, W=W, steps=steps, precision=precision,
                    note=f"sigma redraws={redraws}; droplets={len(drops)}")


def taylor_green(n: int = 64, amp: float = 1e-3, nu: float = 0.1) -> Workload:
    """Single-phase-limit Taylor-Green vortex: N=2 with phase 1 everywhere
    (c_1 = 1), velocity u = A (-cos kx sin ky, sin kx cos ky), k = 2 pi / n."""
    x, y = grid(n, n)
    k = 2.0 * np.pi / n
    u = np.stack([-amp * np.cos(k * x) * np.sin(k * y), amp * np.sin(k * x) * np.cos(k * y)])
    c = np.stack([np.ones((n, n)), np.zeros((n, n))])
    return Workload("taylor_green", 2, n, n, uniform_sigma(2, 1e-3), np.ones(2),
                    np.full(2, nu), c, u, mobility=0.1, tau_phi=0.8, W=4.0)


def cosine_perturbation(n: int = 64, c0: float = 0.05, amp: float = 1e-4,
                        mobility: float = 0.1, sigma: float = 1e-3) -> Workload:
    """N=2, equal densities: c_2 = c0 + amp cos(2 pi x / n), at rest."""
    x, _ = grid(n, n)
    c2 = c0 + amp * np.cos(2.0 * np.pi * x / n)
    return Workload("ch_dispersion", 2, n, n, uniform_sigma(2, sigma), np.ones(2),
                    np.full(2, 0.1), np.stack([1.0 - c2, c2]), None, mobility=mobility,
                    tau_phi=0.8, W=4.0)


def random_smooth(N: int, nx: int, ny: int, seed: int, wall_y: bool = False,
                  amp_u: float = 1e-2, accept=None, W: float = 4.0,
                  unequal: bool = True, sigma_range=(0.5e-3, 2e-3)) -> Workload:
    """Small random test case: N smooth random non-negative fractions that sum
    to one, a smooth random velocity, random tensions (uniform over
    ``sigma_range``; large N needs a narrow range for an SPD mixing matrix),
    densities in [1, 3] and per-phase viscosities (so tau_g varies in
    space)."""
    rng = np.random.default_rng(seed)
    x, y = grid(nx, ny)
    fields = []
    for k in range(N):
        a = np.zeros((ny, nx))
        for _ in range(3):
            kx, ky = rng.integers(0, 3, size=2)
            ph = rng.uniform(0, 2 * np.pi)
            a += rng.uniform(0.2, 1.0) * np.cos(2 * np.pi * (kx * x / nx + ky * y / ny) + ph)
        fields.append(np.exp(1.5 * a))
    tot = sum(fields)
    c = np.stack([f / tot for f in fields[:-1]])
    c = np.concatenate([c, (1.0 - c.sum(axis=0))[None]])
    u = np.zeros((2, ny, nx))
    for d in range(2):
        kx, ky = rng.integers(1, 3, size=2)
        ph = rng.uniform(0, 2 * np.pi)
        u[d] = amp_u * np.sin(2 * np.pi * (kx * x / nx + ky * y / ny) + ph)
    rho = rng.uniform(1.0, 3.0, size=N) if unequal else np.ones(N)
    sigma, _ = draw_sigma(N, seed + 1, *sigma_range, accept=accept, rho=rho)
    mu = rng.uniform(0.05, 0.3, size=N) * rho
    return Workload(f"random_N{N}_{nx}x{ny}", N, nx, ny, sigma, rho, mu, c, u,
                    mobility=float(rng.uniform(0.05, 0.2)), tau_phi=float(rng.uniform(0.7, 1.2)),
                    W=W, wall_y=wall_y, gx=float(rng.uniform(-1e-5, 1e-5)),
                    gy=float(rng.uniform(-1e-5, 1e-5)))


# ---------------------------------------------------------------------------
# Three-dimensional (D3Q15) workloads
# ---------------------------------------------------------------------------

def grid3(nx: int, ny: int, nz: int):
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx].astype(np.float64)
    return x, y, z


def random_smooth3d(N: int, nx: int, ny: int, nz: int, seed: int, wall_z: bool = False,
                    amp_u: float = 1e-2, accept=None, W: float = 4.0,
                    unequal: bool = True) -> Workload:
    """3-D counterpart of random_smooth: N smooth random non-negative
    fractions summing to one, a smooth random velocity (3 components),
    random tensions, densities in [1, 3], per-phase viscosities and a small
    body force."""
    rng = np.random.default_rng(seed)
    x, y, z = grid3(nx, ny, nz)
    fields = []
    for _ in range(N):
        a = np.zeros((nz, ny, nx))
        for _ in range(3):
            kx, ky, kz = rng.integers(0, 3, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            a += rng.uniform(0.2, 1.0) * np.cos(
                2 * np.pi * (kx * x / nx + ky * y / ny + kz * z / nz) + ph)
        fields.append(np.exp(1.5 * a))
    tot = sum(fields)
    c = np.stack([f / tot for f in fields[:-1]])
    c = np.concatenate([c, (1.0 - c.sum(axis=0))[None]])
    u = np.zeros((3, nz, ny, nx))
    for d in range(3):
        kx, ky, kz = rng.integers(1, 3, size=3)
        ph = rng.uniform(0, 2 * np.pi)
        u[d] = amp_u * np.sin(2 * np.pi * (kx * x / nx + ky * y / ny + kz * z / nz) + ph)
    rho = rng.uniform(1.0, 3.0, size=N) if unequal else np.ones(N)
    sigma, _ = draw_sigma(N, seed + 1, accept=accept, rho=rho)
    mu = rng.uniform(0.05, 0.3, size=N) * rho
    return Workload(f"random3d_N{N}_{nx}x{ny}x{nz}", N, nx, ny, sigma, rho, mu, c, u,
                    mobility=float(rng.uniform(0.05, 0.2)), tau_phi=float(rng.uniform(0.7, 1.2)),
                    W=W, gx=float(rng.uniform(-1e-5, 1e-5)), gy=float(rng.uniform(-1e-5, 1e-5)),
                    nz=nz, wall_z=wall_z, gz=float(rng.uniform(-1e-5, 1e-5)))


def static_sphere(n: int = 64, R: float = 16.0, W: float = 4.0, sigma: float = 1e-3,
                  tau_g: float = 1.0, precision: int = 64, steps: int = 2000) -> Workload:
    """3-D counterpart of static_droplet: N=3, a phase-2 sphere of radius R at
    the centre of a periodic n^3 box of phase 1, phase 3 absent, equal
    densities, viscosity for tau_g."""
    x, y, z = grid3(n, n, n)
    r = np.sqrt((x - n / 2.0) ** 2 + (y - n / 2.0) ** 2 + (z - n / 2.0) ** 2)
    c2 = _profile(R - r, W)
    c3 = np.zeros_like(c2)
    nu = (tau_g - 0.5) / 3.0
    return Workload("static_sphere_N3", 3, n, n, uniform_sigma(3, sigma), np.ones(3),
                    np.full(3, nu), np.stack([1.0 - c2, c2, c3]), None, mobility=0.1,
                    tau_phi=0.8, W=W, steps=steps, precision=precision, nz=n)


def droplet_collision3d(side: int = 64, W: float = 4.0, seed: int = BASE_SEED + 6,
                        accept=None, precision: int = 32, steps: int = 2000,
                        speed: float = 0.01) -> Workload:
    """3-D counterpart of droplet_collision: N=4 in a periodic side^3 box;
    phases 2, 3, 4 are spheres of radius 10/64 * side at (0.25, 0.5, 0.4),
    (0.75, 0.5, 0.4) and (0.5, 0.5, 0.8) of the box moving with (+v, 0, 0),
    (-v, 0, 0) and (0, 0, -v); u = sum_d c_d v_d; sigma_kl ~ U[0.5e-3,
    2e-3], rho_1 = 1, rho_2..4 ~ U[1, 3], mu_k = 0.1 rho_k."""
    x, y, z = grid3(side, side, side)
    R = 10.0 * side / 64.0
    centres = [(0.25, 0.5, 0.4, (speed, 0.0, 0.0)), (0.75, 0.5, 0.4, (-speed, 0.0, 0.0)),
               (0.5, 0.5, 0.8, (0.0, 0.0, -speed))]
    cs, u = [], np.zeros((3,) + x.shape)
    for fx, fy, fz, v in centres:
        r = np.sqrt((x - fx * side) ** 2 + (y - fy * side) ** 2 + (z - fz * side) ** 2)
        cd = _profile(R - r, W)
        cs.append(cd)
        for d in range(3):
            u[d] += cd * v[d]
    c = np.stack([1.0 - sum(cs)] + cs)
    rng = np.random.default_rng(seed + 1000)
    rho = np.concatenate([[1.0], rng.uniform(1.0, 3.0, size=3)])
    sigma, redraws = draw_sigma(4, seed, accept=accept, rho=rho)
    return Workload("droplet_collision3d_N4", 4, side, side, sigma, rho, 0.1 * rho, c, u,
                    mobility=0.1, tau_phi=0.8, W=W, steps=steps, precision=precision, nz=side,
                    note=f"sigma redraws={redraws}")


def slabs_and_spheres(side: int = 256, ndrop: int = 64, W: float = 4.0,
                      seed: int = BASE_SEED + 5, accept=None, precision: int = 32,
                      steps: int = 20000, rmin: float = 6.0, rmax: float = 20.0) -> Workload:
    """3-D counterpart of bands_and_droplets: N=5 in a periodic side^3 box;
    slabs of phases 1, 2, 3 of thickness side/4 stacked in z from z = side/8
    (phase 4 fills the rest), plus ``ndrop`` phase-5 spheres with radius ~
    U[rmin, rmax] at seeded, non-overlapping centres (gap >= 2W); sigma_kl ~
    U[0.5e-3, 2e-3], rho_k ~ U[1, 3], mu_k = 0.1 rho_k."""
    z = np.arange(side, dtype=np.float64)[:, None, None]
    h, z0 = side / 4.0, side / 8.0
    slabs = [np.broadcast_to(0.5 * (np.tanh(2.0 * (z - (z0 + b * h)) / W)
                                    - np.tanh(2.0 * (z - (z0 + (b + 1) * h)) / W)),
                             (side, side, side)) for b in range(3)]
    rng = np.random.default_rng(seed)
    drops: List[tuple] = []
    tries = 0
    while len(drops) < ndrop:
        tries += 1
        if tries > 200000:
            raise RuntimeError("could not place spheres")
        r = rng.uniform(rmin, rmax)
        cen = rng.uniform(r + W, side - r - W, size=3)
        if all(np.linalg.norm(cen - np.array(d[:3])) >= r + d[3] + 2 * W for d in drops):
            drops.append((cen[0], cen[1], cen[2], r))
    c5 = np.zeros((side, side, side))
    for xc, yc, zc, r in drops:
        lo = [int(max(0, v - r - 4 * W)) for v in (xc, yc, zc)]
        hi = [int(min(side, v + r + 4 * W + 1)) for v in (xc, yc, zc)]
        zz, yy, xx = np.mgrid[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].astype(np.float64)
        d = r - np.sqrt((xx - xc) ** 2 + (yy - yc) ** 2 + (zz - zc) ** 2)
        c5[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] += _profile(d, W)
    np.minimum(c5, 1.0, out=c5)
    keep = 1.0 - c5
    phases = [s_ * keep for s_ in slabs]
    c4 = 1.0 - phases[0] - phases[1] - phases[2] - c5
    c = np.stack(phases + [c4, c5])
    rng2 = np.random.default_rng(seed + 1000)
    rho = rng2.uniform(1.0, 3.0, size=5)
    sigma, redraws = draw_sigma(5, seed + 7, accept=accept, rho=rho)
    return Workload("slabs_spheres_N5", 5, side, side, sigma, rho, 0.1 * rho, c, None,
                    mobility=0.1, tau_phi=0.8, W=W, steps=steps, precision=precision,
                    nz=side, note=f"sigma redraws={redraws}; spheres={len(drops)}")


# ---------------------------------------------------------------------------
# Serving request stream
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Request:
    rid: int
    arrival: float     # seconds after the stream starts
    N: int
    side: int
    steps: int
    seed: int


def request_stream(n: int = 512, rate: float = 10.0, seed: int = BASE_SEED + 5,
                   side_lo: int = 64, side_hi: int = 1024, steps_lo: int = 1000,
                   steps_hi: int = 20000) -> List[Request]:
    """Poisson arrivals at ``rate`` per second; N uniform in {3,4,5}; side
    log-uniform on [side_lo, side_hi] rounded to a multiple of 16; steps
    uniform on [steps_lo, steps_hi]."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        N = int(rng.integers(3, 6))
        side = math.exp(rng.uniform(math.log(side_lo), math.log(side_hi)))
        side = int(max(side_lo, min(side_hi, 16 * round(side / 16))))
        steps = int(rng.integers(steps_lo, steps_hi + 1))
        out.append(Request(i, t, N, side, steps, seed * 1000 + i))
    return out


def request_workload(req: Request, accept=None) -> Workload:
    """The layout of one serving request: a static droplet for N=3, a scaled
    droplet collision for N=4, scaled bands and droplets for N=5."""
    if req.N == 3:
        w = static_droplet(req.side, req.side, R=req.side / 4.0, precision=32,
                           steps=req.steps)
    elif req.N == 4:
        w = droplet_collision(req.side, seed=req.seed, accept=accept, precision=32,
                              steps=req.steps)
    else:
        nd = int(max(4, round(64 * req.side ** 2 / 2048 ** 2)))
        rmax = max(6.0, min(40.0, req.side / 12.0))
        rmin = min(10.0, rmax / 2.0)
        w = bands_and_droplets(req.side, ndrop=nd, seed=req.seed, accept=accept,
                               precision=32, steps=req.steps, rmin=rmin, rmax=rmax)
    w.name = f"req{req.rid}_{w.name}_{req.side}"
    return w
