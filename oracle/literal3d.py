"""Second, independent CPU transcription of the N-phase LB step on the D3Q15
lattice (NumPy, FP64).

TEST INFRASTRUCTURE ONLY.  It cross-checks the C oracle's 3-D version
(nplbm_oracle3d.c) on tiny grids.  Like the 2-D transcription it works on
whole arrays: np.roll for shifts, all fifteen NS populations kept (including
g_0 with the constant rho_0 of eq:25), mirror ghost planes padded next to z
walls, streaming by rolling.  The lambda solve of eq:N14-N16 is the 2-D
transcription's (it does not depend on the lattice).

Equations: eq:N1, eq:N12, eq:N17, eq:N18, eq:N36 (closure), eq:N31a/b on
D3Q15 (stencils), eq:24, eq:25, eq:N20_1, eq:N21_1, eq:N22_1, eq:N23 (NS
part), eq:N24-N28, eq:N30 (CH part); D3Q15 velocities and weights of
Sec. 3.1.
"""
from __future__ import annotations

import numpy as np

from .literal import LiteralSim

E = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [-1, 0, 0], [0, -1, 0], [0, 0, -1],
              [1, 1, 1], [1, 1, -1], [1, -1, 1], [-1, 1, 1], [-1, -1, -1], [-1, -1, 1],
              [-1, 1, -1], [1, -1, -1]])
WGT = np.array([2 / 9] + [1 / 9] * 6 + [1 / 72] * 8)
CS2 = 1.0 / 3.0
Q = 15


def _b(v):
    """broadcast a per-phase vector over (z, y, x)"""
    return np.asarray(v)[:, None, None, None]


class LiteralSim3D:
    def __init__(self, N, nx, ny, nz, sigma, rho, mu, mobility=0.1, tau_phi=0.8, W=4.0,
                 wall_z=False, gx=0.0, gy=0.0, gz=0.0, rho0=1.0):
        self.N, self.nx, self.ny, self.nz = N, nx, ny, nz
        two = LiteralSim(N, 4, 4, sigma, rho, mu, mobility, tau_phi, W)
        self.lam, self.K = two.lam, two.K
        self.rt = np.asarray(rho, float) * np.ones(N)
        self.mt = np.asarray(mu, float) * np.ones(N)
        self.m = np.asarray(mobility, float) * np.ones(N - 1)
        self.tau = np.asarray(tau_phi, float) * np.ones(N - 1)
        self.wall = bool(wall_z)
        self.G = np.array([gx, gy, gz], float)
        self.rho0 = rho0
        self.gam = 1.0 / self.rt
        self.Gam = self.gam.sum()
        self.eta_i = self.m / (CS2 * (self.tau - 0.5))          # eq:N30
        self.a = 0.5 * (self.rt[:-1] + self.rt[-1])
        self.b = 0.5 * (self.rt[:-1] - self.rt[-1])
        self.opp = [int(np.nonzero((E == -E[k]).all(axis=1))[0][0]) for k in range(Q)]

    # zeta(x + d): periodic in x, y; periodic or mirror ghosts in z
    def shift(self, f, d):
        g = np.roll(np.roll(f, -d[0], axis=-1), -d[1], axis=-2)
        if not self.wall:
            return np.roll(g, -d[2], axis=-3)
        pad = np.concatenate([g[..., :1, :, :], g, g[..., -1:, :, :]], axis=-3)
        return pad[..., 1 + d[2]: 1 + d[2] + self.nz, :, :]

    def grad(self, f):                                           # eq:N31a
        out = np.zeros((3,) + f.shape)
        for k in range(1, Q):
            diff = self.shift(f, E[k]) - self.shift(f, -E[k])
            for a in range(3):
                out[a] += WGT[k] * E[k, a] * diff / (2 * CS2)
        return out

    def lap(self, f):                                            # eq:N31b
        out = np.zeros(f.shape)
        for k in range(1, Q):
            out += WGT[k] * (self.shift(f, E[k]) - 2 * f + self.shift(f, -E[k])) / CS2
        return out

    def closure(self, phi):                                      # eq:N18
        vphi = _b(self.b) + _b(self.a) * phi                     # eq:N12
        rho_i = np.empty((self.N,) + phi.shape[1:])
        for i in range(self.N):
            rho_i[i] = 1.0 / self.Gam
            for j in range(self.N - 1):
                rho_i[i] += ((i == j) - self.gam[j] / self.Gam) * vphi[j]
        return _b(self.gam) * rho_i, rho_i.sum(axis=0)

    def hfun(self, c):                                           # eq:N17
        w = c * (1 - c) * (1 - 2 * c)
        out = np.zeros((self.N - 1,) + c.shape[1:])
        for i in range(self.N - 1):
            for k in range(self.N):
                out[i] += (self.gam[k] * (k == i) - self.gam[k] * self.gam[i] / self.Gam) * w[k]
            out[i] *= self.a[i]
        return out

    def chem(self, phi, c):
        lp = np.stack([self.lap(phi[j]) for j in range(self.N - 1)])
        return -np.einsum("ij,j...->i...", self.lam, lp) + self.K * self.hfun(c)

    def heq(self, phi, Cp, u):                                   # eq:N25
        out = np.empty((self.N - 1, Q) + phi.shape[1:])
        for k in range(Q):
            cu = sum(E[k, a] * u[a] for a in range(3))
            if k == 0:
                out[:, 0] = phi + (WGT[0] - 1) * _b(self.eta_i) * Cp
            else:
                out[:, k] = WGT[k] * _b(self.eta_i) * Cp + WGT[k] * phi * cu / CS2
        return out

    def geq(self, rho, p, u):                                    # eq:25
        out = np.empty((Q,) + rho.shape)
        uu = (u ** 2).sum(axis=0)
        for k in range(Q):
            cu = sum(E[k, a] * u[a] for a in range(3))
            s = WGT[k] * (cu / CS2 + cu ** 2 / (2 * CS2 ** 2) - uu / (2 * CS2))
            out[k] = p / CS2 * WGT[k] + rho * s
            if k == 0:
                out[k] += self.rho0 - p / CS2
        return out

    def init(self, c, u=None):
        c = np.asarray(c, float)
        sh = (self.nz, self.ny, self.nx)
        u = np.zeros((3,) + sh) if u is None else np.asarray(u, float)
        phi = (_b(self.rt[:-1]) * c[:-1] - self.rt[-1] * c[-1] - _b(self.b)) / _b(self.a)
        cc, rho = self.closure(phi)
        self.h = self.heq(phi, self.chem(phi, cc), u)
        self.g = self.geq(rho, np.zeros_like(rho), u)
        self.pphi, self.pu = phi.copy(), u.copy()

    def macro_all(self):
        phi = self.h.sum(axis=1)                                 # eq:N28
        c, rho = self.closure(phi)
        Cp = self.chem(phi, c)
        gphi = np.stack([self.grad(phi[i]) for i in range(self.N - 1)])
        gC = np.stack([self.grad(Cp[i]) for i in range(self.N - 1)])
        grho = self.grad(rho)
        F = np.einsum("i...,id...->d...", Cp, gphi) + rho[None] * self.G[:, None, None, None]
        coef = (1 - self.N * self.gam[:-1] / self.Gam) * self.a * self.m
        J = -np.einsum("i,id...->d...", coef, gC)
        mom = np.einsum("kd,k...->d...", E.astype(float), self.g)
        u = (mom + 0.5 * F) / rho                                # eq:N22_1
        s0 = WGT[0] * (-(u ** 2).sum(axis=0) / (2 * CS2))
        p = CS2 / (1 - WGT[0]) * (self.g[1:].sum(axis=0) + 0.5 * (u * grho).sum(axis=0)
                                  + rho * s0)                    # eq:N23
        taug = 0.5 + np.einsum("k,k...->...", self.mt, c) / (rho * CS2)
        return dict(phi=phi, c=c, rho=rho, C=Cp, F=F, J=J, grho=grho, u=u, p=p, taug=taug)

    def step(self, n=1):
        for _ in range(n):
            m = self.macro_all()
            u, rho, p, tg = m["u"], m["rho"], m["p"], m["taug"]
            F, grho, J = m["F"], m["grho"], m["J"]
            geq = self.geq(rho, p, u)
            T = np.empty((3, 3) + rho.shape)
            for al in range(3):
                for be in range(3):
                    T[al, be] = (u[al] * F[be] + F[al] * u[be] +
                                 CS2 * (u[al] * grho[be] + grho[al] * u[be]) +
                                 J[al] * u[be] / (tg - 0.5))
            gs = np.empty_like(self.g)
            for k in range(Q):
                ck = E[k].astype(float)
                con = sum((ck[al] * ck[be] - CS2 * (al == be)) * T[al, be]
                          for al in range(3) for be in range(3))
                Gk = WGT[k] * ((u * grho).sum(axis=0) + sum(ck[a] * F[a] for a in range(3)) / CS2
                               + con / (2 * CS2 ** 2))           # eq:N20_1
                gs[k] = self.g[k] - (self.g[k] - geq[k]) / tg + (1 - 1 / (2 * tg)) * Gk
            heq = self.heq(m["phi"], m["C"], u)
            dpu = m["phi"][:, None] * u[None] - self.pphi[:, None] * self.pu[None]   # eq:N27
            hs = np.empty_like(self.h)
            for k in range(Q):
                R = (_b(1 - 1 / (2 * self.tau)) * WGT[k] *
                     sum(E[k, a] * dpu[:, a] for a in range(3)) / CS2)              # eq:N26
                hs[:, k] = self.h[:, k] - (self.h[:, k] - heq[:, k]) / _b(self.tau) + R
            self.pphi, self.pu = m["phi"].copy(), u.copy()
            self.h = self._stream(hs)
            self.g = self._stream(gs[None])[0]

    def _stream(self, fs):
        out = np.empty_like(fs)
        for k in range(Q):
            dx, dy, dz = E[k]
            moved = np.roll(np.roll(np.roll(fs[:, k], dx, axis=-1), dy, axis=-2), dz, axis=-3)
            if self.wall and dz != 0:
                if dz > 0:
                    moved[:, 0] = 0.0
                else:
                    moved[:, -1] = 0.0
            out[:, k] = moved
        if self.wall:
            for k in range(Q):
                dz = E[k, 2]
                if dz > 0:      # leaving through the top wall
                    out[:, self.opp[k], -1] = fs[:, k, -1]
                elif dz < 0:    # leaving through the bottom wall
                    out[:, self.opp[k], 0] = fs[:, k, 0]
        return out

    def macro(self):
        m = self.macro_all()
        return m["c"], m["u"], m["p"]
