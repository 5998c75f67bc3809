"""FP64 CPU oracle for the N-phase phase-field LB model (arXiv:1904.12553).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The oracle shares no code with the
GPU library and the GPU library never calls it.

Two independent CPU implementations live here:

* ``OracleSim`` -- ctypes wrapper over ``nplbm_oracle.c`` (plain C, FP64);
* ``OracleSim3D`` -- the same model on the D3Q15 lattice, ``nplbm_oracle3d.c``;
* ``oracle.literal`` -- a NumPy transcription over whole arrays that keeps all
  nine NS populations (including g_0 and rho_0), used to cross-check the C
  oracle on tiny grids.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


ORC_OK, ORC_EINVAL, ORC_ENOTSPD, ORC_ENOMEM = 0, -1, -2, -3


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        srcs = [os.path.join(HERE, f) for f in ("nplbm_oracle.c", "nplbm_oracle3d.c")]
        if not os.path.exists(path) or os.path.getmtime(path) < max(map(os.path.getmtime, srcs)):
            from . import build_oracle as _b
            _b.build()
        lib = ctypes.CDLL(path)
        d, i, l, vp = ctypes.c_double, ctypes.c_int, ctypes.c_long, ctypes.c_void_p
        P = ctypes.POINTER(ctypes.c_double)
        lib.orc_create.argtypes = [i, i, i, i, i, i, P, P, P, P, P, d, d, d, d,
                                   ctypes.POINTER(vp)]
        lib.orc_create.restype = i
        lib.orc_free.argtypes = [vp]
        lib.orc_init.argtypes = [vp, P, P]
        lib.orc_step.argtypes = [vp, l]
        lib.orc_macro.argtypes = [vp, P, P, P]
        lib.orc_fields.argtypes = [vp, P, P, P, P, P, P, P]
        lib.orc_mass.argtypes = [vp, P]
        lib.orc_time.argtypes = [vp]
        lib.orc_time.restype = l
        lib.orc_get_state.argtypes = [vp, P, P, P, P]
        lib.orc_set_state.argtypes = [vp, P, P, P, P]
        lib.orc_lambda.argtypes = [vp, P, P, P, P]
        lib.orc_Lvec.argtypes = [vp, i, i, i]
        lib.orc_Lvec.restype = d
        lib.orc_closure.argtypes = [vp, P, P, P]
        lib.orc_hbulk.argtypes = [vp, P, P]
        lib.orc_node_dists.argtypes = [vp] + [d] * 11 + [P, P]
        lib.orc_node_heq.argtypes = [vp, i, d, d, d, d, P]
        lib.orc_stencils.argtypes = [vp, P, P, P]
        lib.orc3_create.argtypes = [i, i, i, i, i, P, P, P, P, P, d, d, d, d, d,
                                    ctypes.POINTER(vp)]
        lib.orc3_create.restype = i
        lib.orc3_free.argtypes = [vp]
        lib.orc3_init.argtypes = [vp, P, P]
        lib.orc3_step.argtypes = [vp, l]
        lib.orc3_macro.argtypes = [vp, P, P, P]
        lib.orc3_fields.argtypes = [vp, P, P, P, P, P, P]
        lib.orc3_mass.argtypes = [vp, P]
        lib.orc3_time.argtypes = [vp]
        lib.orc3_time.restype = l
        lib.orc3_get_state.argtypes = [vp, P, P, P, P]
        lib.orc3_node_dists.argtypes = [vp, d, d, P, P, P, P, d, P, P]
        lib.orc3_node_heq.argtypes = [vp, i, d, d, P, P]
        lib.orc3_stencils.argtypes = [vp, P, P, P]
        _LIB = lib
    return _LIB


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _arr(x, n):
    a = np.ascontiguousarray(np.broadcast_to(np.asarray(x, dtype=np.float64), (n,)))
    return a


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle error {code}")
        self.code = code


class OracleSim:
    """One simulation domain in the FP64 oracle.

    Parameters follow the paper's problem statement: N phases with pairwise
    surface tensions ``sigma`` (N x N, symmetric), densities ``rho`` and
    dynamic viscosities ``mu`` (N each), CH mobility ``mobility`` and
    relaxation time ``tau_phi`` (scalars or N-1 values), interface width
    ``W`` (= 2 sqrt(2) eta), body-force acceleration ``(gx, gy)``.
    ``force_form`` 0 is the total-force distribution of eq:N20_1, 1 the one
    of Remark 1 (Sec. 3.1) with F = -div(J~ u) + F_s + G.
    """

    def __init__(self, N, nx, ny, sigma, rho, mu, mobility=0.1, tau_phi=0.8,
                 W=4.0, wall_y=False, gx=0.0, gy=0.0, rho0=1.0, grad_scheme=0, force_form=0):
        lib = _lib()
        self.N, self.nx, self.ny = int(N), int(nx), int(ny)
        sig = np.ascontiguousarray(np.asarray(sigma, dtype=np.float64).reshape(N, N))
        r = _arr(rho, N)
        m = _arr(mu, N)
        mob = _arr(mobility, N - 1)
        tp = _arr(tau_phi, N - 1)
        h = ctypes.c_void_p()
        rc = lib.orc_create(self.N, self.nx, self.ny, int(bool(wall_y)), int(grad_scheme),
                            int(force_form), _p(sig), _p(r), _p(m), _p(mob), _p(tp), float(W),
                            float(gx), float(gy), float(rho0), ctypes.byref(h))
        if rc != 0:
            raise OracleError(rc)
        self._h = h
        self._keep = (sig, r, m, mob, tp)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _lib().orc_free(h)
            self._h = None

    @property
    def n(self):
        return self.nx * self.ny

    def init(self, c, u=None):
        c = np.ascontiguousarray(c, dtype=np.float64).reshape(self.N, self.ny, self.nx)
        uu = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(2, self.ny, self.nx)
        _lib().orc_init(self._h, _p(c), _p(uu))

    def step(self, nsteps=1):
        _lib().orc_step(self._h, int(nsteps))

    @property
    def time(self):
        return _lib().orc_time(self._h)

    def macro(self):
        c = np.empty((self.N, self.ny, self.nx))
        u = np.empty((2, self.ny, self.nx))
        p = np.empty((self.ny, self.nx))
        _lib().orc_macro(self._h, _p(c), _p(u), _p(p))
        return c, u, p

    def fields(self):
        n1 = self.N - 1
        sh = (self.ny, self.nx)
        out = dict(phi=np.empty((n1,) + sh), rho=np.empty(sh), C=np.empty((n1,) + sh),
                   F=np.empty((2,) + sh), J=np.empty((2,) + sh), grho=np.empty((2,) + sh),
                   taug=np.empty(sh))
        _lib().orc_fields(self._h, _p(out["phi"]), _p(out["rho"]), _p(out["C"]), _p(out["F"]),
                          _p(out["J"]), _p(out["grho"]), _p(out["taug"]))
        return out

    def mass(self):
        m = np.empty(self.N)
        _lib().orc_mass(self._h, _p(m))
        return m

    def get_state(self):
        n1 = self.N - 1
        sh = (self.ny, self.nx)
        h = np.empty((n1, 9) + sh)
        g = np.empty((9,) + sh)
        pp = np.empty((n1,) + sh)
        pu = np.empty((2,) + sh)
        _lib().orc_get_state(self._h, _p(h), _p(g), _p(pp), _p(pu))
        return h, g, pp, pu

    def set_state(self, h=None, g=None, pphi=None, pu=None):
        c = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)
        h, g, pphi, pu = c(h), c(g), c(pphi), c(pu)
        _lib().orc_set_state(self._h, _p(h), _p(g), _p(pphi), _p(pu))

    # ---- node-level pieces ----
    def lam(self):
        n1 = self.N - 1
        lam = np.empty((n1, n1))
        b2, K, eta = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _lib().orc_lambda(self._h, _p(lam), ctypes.byref(b2), ctypes.byref(K), ctypes.byref(eta))
        return lam, b2.value, K.value, eta.value

    def Lvec(self, k, l):
        return np.array([_lib().orc_Lvec(self._h, k, l, i) for i in range(1, self.N)])

    def closure(self, phi):
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        c = np.empty(self.N)
        r = np.empty(1)
        _lib().orc_closure(self._h, _p(phi), _p(c), _p(r))
        return c, r[0]

    def hbulk(self, phi):
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        h = np.empty(self.N - 1)
        _lib().orc_hbulk(self._h, _p(phi), _p(h))
        return h

    def node_dists(self, rho, p, u, F, grho, J, taug):
        geq = np.empty(9)
        G = np.empty(9)
        _lib().orc_node_dists(self._h, rho, p, u[0], u[1], F[0], F[1], grho[0], grho[1],
                              J[0], J[1], taug, _p(geq), _p(G))
        return geq, G

    def node_heq(self, i, phi, C, u):
        heq = np.empty(9)
        _lib().orc_node_heq(self._h, int(i), phi, C, u[0], u[1], _p(heq))
        return heq

    def stencils(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.ny, self.nx)
        lap = np.empty((self.ny, self.nx))
        g = np.empty((2, self.ny, self.nx))
        _lib().orc_stencils(self._h, _p(f), _p(lap), _p(g))
        return lap, g


class OracleSim3D:
    """One 3-D domain (D3Q15 lattice of Sec. 3.1) in the FP64 oracle.

    Same parameters as ``OracleSim`` plus ``nz``; x and y are periodic, z is
    periodic or bounded by halfway bounce-back walls (``wall_z``); the body
    force is rho (gx, gy, gz).  Fields have shape (.., nz, ny, nx)."""

    def __init__(self, N, nx, ny, nz, sigma, rho, mu, mobility=0.1, tau_phi=0.8, W=4.0,
                 wall_z=False, gx=0.0, gy=0.0, gz=0.0, rho0=1.0):
        lib = _lib()
        self.N, self.nx, self.ny, self.nz = int(N), int(nx), int(ny), int(nz)
        sig = np.ascontiguousarray(np.asarray(sigma, dtype=np.float64).reshape(N, N))
        r, m = _arr(rho, N), _arr(mu, N)
        mob, tp = _arr(mobility, N - 1), _arr(tau_phi, N - 1)
        h = ctypes.c_void_p()
        rc = lib.orc3_create(self.N, self.nx, self.ny, self.nz, int(bool(wall_z)), _p(sig),
                             _p(r), _p(m), _p(mob), _p(tp), float(W), float(gx), float(gy),
                             float(gz), float(rho0), ctypes.byref(h))
        if rc != 0:
            raise OracleError(rc)
        self._h = h
        self._keep = (sig, r, m, mob, tp)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _lib().orc3_free(h)
            self._h = None

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def init(self, c, u=None):
        c = np.ascontiguousarray(c, dtype=np.float64).reshape((self.N,) + self.shape)
        uu = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(
            (3,) + self.shape)
        _lib().orc3_init(self._h, _p(c), _p(uu))

    def step(self, nsteps=1):
        _lib().orc3_step(self._h, int(nsteps))

    @property
    def time(self):
        return _lib().orc3_time(self._h)

    def macro(self):
        c = np.empty((self.N,) + self.shape)
        u = np.empty((3,) + self.shape)
        p = np.empty(self.shape)
        _lib().orc3_macro(self._h, _p(c), _p(u), _p(p))
        return c, u, p

    def fields(self):
        sh = self.shape
        out = dict(phi=np.empty((self.N - 1,) + sh), rho=np.empty(sh),
                   C=np.empty((self.N - 1,) + sh), F=np.empty((3,) + sh),
                   J=np.empty((3,) + sh), grho=np.empty((3,) + sh))
        _lib().orc3_fields(self._h, _p(out["phi"]), _p(out["rho"]), _p(out["C"]),
                           _p(out["F"]), _p(out["J"]), _p(out["grho"]))
        return out

    def mass(self):
        m = np.empty(self.N)
        _lib().orc3_mass(self._h, _p(m))
        return m

    def get_state(self):
        sh = self.shape
        h = np.empty((self.N - 1, 15) + sh)
        g = np.empty((15,) + sh)
        pp = np.empty((self.N - 1,) + sh)
        pu = np.empty((3,) + sh)
        _lib().orc3_get_state(self._h, _p(h), _p(g), _p(pp), _p(pu))
        return h, g, pp, pu

    def node_dists(self, rho, p, u, F, grho, J, taug):
        geq, G = np.empty(15), np.empty(15)
        a = [np.ascontiguousarray(v, dtype=np.float64) for v in (u, F, grho, J)]
        _lib().orc3_node_dists(self._h, float(rho), float(p), _p(a[0]), _p(a[1]), _p(a[2]),
                               _p(a[3]), float(taug), _p(geq), _p(G))
        return geq, G

    def node_heq(self, i, phi, C, u):
        heq = np.empty(15)
        uu = np.ascontiguousarray(u, dtype=np.float64)
        _lib().orc3_node_heq(self._h, int(i), float(phi), float(C), _p(uu), _p(heq))
        return heq

    def stencils(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.shape)
        lap = np.empty(self.shape)
        g = np.empty((3,) + self.shape)
        _lib().orc3_stencils(self._h, _p(f), _p(lap), _p(g))
        return lap, g


def build():
    from . import build_oracle as _b
    return _b.build()
