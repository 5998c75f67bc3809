"""Second, independent CPU transcription of the N-phase LB step (NumPy, FP64).

TEST INFRASTRUCTURE ONLY.  It exists to cross-check the C oracle on tiny
grids: it is written from the paper's equations directly over whole arrays
(np.roll for shifts), keeps all nine NS populations including g_0 and the
constant rho_0 of eq:25, pads fields with mirror ghost rows next to walls and
streams by rolling, so that it shares neither structure nor helpers with the
C oracle.

Equations: eq:N1, eq:N12, eq:N14-N18, eq:N36 (setup and closure);
eq:N31a/b (stencils), eq:N40 (mixed gradient, two-hop term read as
negative); eq:24, eq:25, eq:N20_1 or the force distribution of Remark 1
(Sec. 3.1, with div(J~ u) taken over J~ of the step and the stored u of the
previous step), eq:N21_1, eq:N22_1, eq:N23 (NS part); eq:N24-N28, eq:N30
(CH part).
"""
from __future__ import annotations

import numpy as np

C = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]])
WGT = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
OPP = [0, 3, 4, 1, 2, 7, 8, 5, 6]
CS2 = 1.0 / 3.0


class LiteralSim:
    def __init__(self, N, nx, ny, sigma, rho, mu, mobility=0.1, tau_phi=0.8, W=4.0,
                 wall_y=False, gx=0.0, gy=0.0, rho0=1.0, grad_scheme=0, force_form=0):
        self.N, self.nx, self.ny = N, nx, ny
        self.grad_scheme = int(grad_scheme)
        self.force_form = int(force_form)
        self.sig = np.asarray(sigma, float).reshape(N, N)
        self.rt = np.asarray(rho, float) * np.ones(N)
        self.mt = np.asarray(mu, float) * np.ones(N)
        self.m = np.asarray(mobility, float) * np.ones(N - 1)
        self.tau = np.asarray(tau_phi, float) * np.ones(N - 1)
        self.wall = bool(wall_y)
        self.G = np.array([gx, gy], float)
        self.rho0 = rho0
        self.eta = W / (2 * np.sqrt(2))
        self.gam = 1.0 / self.rt
        self.Gam = self.gam.sum()
        smin = min(self.sig[k, l] for k in range(N) for l in range(k + 1, N))
        self.beta2 = 3 * np.sqrt(2) * smin * self.eta          # eq:N36
        self.K = self.beta2 / self.eta ** 2
        self.lam = self._lambda()
        self.eta_i = self.m / (CS2 * (self.tau - 0.5))          # eq:N30
        self.a = 0.5 * (self.rt[:-1] + self.rt[-1])
        self.b = 0.5 * (self.rt[:-1] - self.rt[-1])

    # eq:N14-N16 solved with numpy's dense solver
    def _lambda(self):
        N = self.N
        r = self.rt
        unk = [(i, j) for i in range(N - 1) for j in range(i, N - 1)]
        rows, rhs = [], []
        for k in range(N):
            for l in range(k + 1, N):
                L = np.zeros(N - 1)
                for i in range(N - 1):
                    if l == N - 1:
                        L[i] = 1.0 if i == k else r[N - 1] / (r[i] + r[N - 1])
                    else:
                        L[i] = (r[k] / (r[k] + r[N - 1]) if i == k else
                                -r[l] / (r[l] + r[N - 1]) if i == l else 0.0)
                rows.append([L[i] * L[j] * (1 if i == j else 2) for i, j in unk])
                rhs.append(4.5 * self.eta ** 2 / self.beta2 * self.sig[k, l] ** 2)
        x = np.linalg.solve(np.array(rows), np.array(rhs))
        lam = np.zeros((N - 1, N - 1))
        for (i, j), v in zip(unk, x):
            lam[i, j] = lam[j, i] = v
        return lam

    # shifted copy zeta(x + d): periodic in x; periodic or mirror ghosts in y
    def shift(self, f, dx, dy):
        g = np.roll(f, -dx, axis=-1)
        if not self.wall:
            return np.roll(g, -dy, axis=-2)
        pad = np.concatenate([g[..., 1::-1, :], g, g[..., :-3:-1, :]], axis=-2)
        return pad[..., 2 + dy: 2 + dy + self.ny, :]

    def grad(self, f):                                           # eq:N31a
        if self.grad_scheme == 1:
            return self.grad_mixed(f)
        out = np.zeros((2,) + f.shape)
        for k in range(1, 9):
            d = self.shift(f, *C[k]) - self.shift(f, *(-C[k]))
            out[0] += WGT[k] * C[k, 0] * d / (2 * CS2)
            out[1] += WGT[k] * C[k, 1] * d / (2 * CS2)
        return out

    def grad_mixed(self, f):                                     # eq:N40
        out = np.zeros((2,) + f.shape)
        for k in range(1, 9):
            cx, cy = C[k]
            d = (-self.shift(f, 2 * cx, 2 * cy) + 5 * self.shift(f, cx, cy) - 3 * f
                 - self.shift(f, -cx, -cy))
            out[0] += WGT[k] * cx * d / (4 * CS2)
            out[1] += WGT[k] * cy * d / (4 * CS2)
        return out

    def lap(self, f):                                            # eq:N31b
        out = np.zeros(f.shape)
        for k in range(1, 9):
            out += WGT[k] * (self.shift(f, *C[k]) - 2 * f + self.shift(f, *(-C[k]))) / CS2
        return out

    def closure(self, phi):                                      # eq:N18
        vphi = self.b[:, None, None] + self.a[:, None, None] * phi     # eq:N12
        rho_i = np.empty((self.N,) + phi.shape[1:])
        for i in range(self.N):
            rho_i[i] = 1.0 / self.Gam
            for j in range(self.N - 1):
                rho_i[i] += ((i == j) - self.gam[j] / self.Gam) * vphi[j]
        c = self.gam[:, None, None] * rho_i
        rho = rho_i.sum(axis=0)
        return c, rho

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
        return -np.einsum("ij,jyx->iyx", self.lam, lp) + self.K * self.hfun(c)

    def heq(self, phi, Cp, u):                                   # eq:N25
        out = np.empty((self.N - 1, 9) + phi.shape[1:])
        for k in range(9):
            cu = C[k, 0] * u[0] + C[k, 1] * u[1]
            if k == 0:
                out[:, 0] = phi + (WGT[0] - 1) * self.eta_i[:, None, None] * Cp
            else:
                out[:, k] = WGT[k] * self.eta_i[:, None, None] * Cp + WGT[k] * phi * cu / CS2
        return out

    def geq(self, rho, p, u):                                    # eq:25
        out = np.empty((9,) + rho.shape)
        uu = u[0] ** 2 + u[1] ** 2
        for k in range(9):
            cu = C[k, 0] * u[0] + C[k, 1] * u[1]
            s = WGT[k] * (cu / CS2 + cu ** 2 / (2 * CS2 ** 2) - uu / (2 * CS2))
            out[k] = p / CS2 * WGT[k] + rho * s
            if k == 0:
                out[k] += self.rho0 - p / CS2
        return out

    def init(self, c, u=None):
        c = np.asarray(c, float)
        u = np.zeros((2, self.ny, self.nx)) if u is None else np.asarray(u, float)
        rN = self.rt[-1]
        phi = (self.rt[:-1, None, None] * c[:-1] - rN * c[-1] - self.b[:, None, None]) / \
            self.a[:, None, None]
        cc, rho = self.closure(phi)
        Cp = self.chem(phi, cc)
        self.h = self.heq(phi, Cp, u)
        self.g = self.geq(rho, np.zeros_like(rho), u)
        self.pphi, self.pu = phi.copy(), u.copy()

    def macro_all(self):
        phi = self.h.sum(axis=1)                                 # eq:N28
        c, rho = self.closure(phi)
        Cp = self.chem(phi, c)
        gphi = np.stack([self.grad(phi[i]) for i in range(self.N - 1)])    # (N-1,2,..)
        gC = np.stack([self.grad(Cp[i]) for i in range(self.N - 1)])
        grho = self.grad(rho)
        F = np.einsum("iyx,idyx->dyx", Cp, gphi) + rho[None] * self.G[:, None, None]
        coef = (1 - self.N * self.gam[:-1] / self.Gam) * self.a * self.m
        J = -np.einsum("i,idyx->dyx", coef, gC)
        if self.force_form == 1:
            F -= self.flux_divergence(J, self.pu)
        mom = np.einsum("kd,kyx->dyx", C.astype(float), self.g)
        u = (mom + 0.5 * F) / rho                                # eq:N22_1
        uu = u[0] ** 2 + u[1] ** 2
        s0 = WGT[0] * (-uu / (2 * CS2))
        p = CS2 / (1 - WGT[0]) * (self.g[1:].sum(axis=0) + 0.5 * (u * grho).sum(axis=0) + rho * s0)
        taug = self.tau_g(c, rho)
        return dict(phi=phi, c=c, rho=rho, C=Cp, F=F, J=J, grho=grho, u=u, p=p, taug=taug)

    def step(self, n=1):
        for _ in range(n):
            m = self.macro_all()
            u, rho, p, tg = m["u"], m["rho"], m["p"], m["taug"]
            F, grho, J = m["F"], m["grho"], m["J"]
            geq = self.geq(rho, p, u)
            gs = np.empty_like(self.g)
            for k in range(9):
                ck = C[k].astype(float)
                # (c c - cs^2 I) : T / (2 cs^4), T = uF + Fu + cs^2(u grho + grho u) + J u/(tau-1/2)
                T = np.empty((2, 2) + rho.shape)
                for al in range(2):
                    for be in range(2):
                        T[al, be] = (u[al] * F[be] + F[al] * u[be] + CS2 * (u[al] * grho[be] +
                                     grho[al] * u[be]) +
                                     (J[al] * u[be] / (tg - 0.5) if self.force_form == 0 else 0.0))
                con = sum((ck[al] * ck[be] - CS2 * (al == be)) * T[al, be]
                          for al in range(2) for be in range(2))
                Gk = WGT[k] * ((u * grho).sum(axis=0) + (ck[0] * F[0] + ck[1] * F[1]) / CS2 +
                               con / (2 * CS2 ** 2))
                gs[k] = self.g[k] - (self.g[k] - geq[k]) / tg + (1 - 1 / (2 * tg)) * Gk
            heq = self.heq(m["phi"], m["C"], u)
            dpu = self.flux_rate(m["phi"], u)
            hs = np.empty_like(self.h)
            for k in range(9):
                R = ((1 - 1 / (2 * self.tau))[:, None, None] * WGT[k] *
                     (C[k, 0] * dpu[:, 0] + C[k, 1] * dpu[:, 1]) / CS2)
                hs[:, k] = self.h[:, k] - (self.h[:, k] - heq[:, k]) / self.tau[:, None, None] + R
            self.pphi, self.pu = m["phi"].copy(), u.copy()
            self.h = self._stream(hs)
            self.g = self._stream(gs[None])[0]

    # The three pieces below are separate methods so that a test can swap in
    # a deliberately wrong reading and show that the pins reject it.
    def flux_rate(self, phi, u):
        """eq:N27: backward-Euler d_t(phi_i u) = phi_i u - phi_i(prev) u(prev),
        shape (N-1, 2, ny, nx)."""
        return phi[:, None] * u[None] - self.pphi[:, None] * self.pu[None]

    def tau_g(self, c, rho):
        """eq:N21_1 with the local dynamic viscosity mu = sum_k mu~_k c_k."""
        mu = np.einsum("k,kyx->yx", self.mt, c)
        return 0.5 + mu / (rho * CS2)

    def flux_divergence(self, J, u):
        """Remark 1: component a of div(J~ u) is sum_b d_b (J~_b u_a)."""
        return np.stack([sum(self.grad(J[b] * u[a])[b] for b in range(2)) for a in range(2)])

    def _stream(self, fs):
        out = np.empty_like(fs)
        for k in range(9):
            dx, dy = C[k]
            moved = np.roll(np.roll(fs[:, k], dx, axis=-1), dy, axis=-2)
            if self.wall and dy != 0:
                # rows that would wrap are bounced back into the opposite direction
                if dy > 0:
                    moved[:, 0, :] = 0.0
                else:
                    moved[:, -1, :] = 0.0
            out[:, k] = moved
        if self.wall:
            for k in range(9):
                dy = C[k, 1]
                if dy > 0:      # populations leaving through the top wall
                    out[:, OPP[k], -1, :] = fs[:, k, -1, :]
                elif dy < 0:    # leaving through the bottom wall
                    out[:, OPP[k], 0, :] = fs[:, k, 0, :]
        return out

    def macro(self):
        m = self.macro_all()
        return m["c"], m["u"], m["p"]
