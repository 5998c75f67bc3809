"""Thin ctypes binding of libnplbm.so (C ABI declared in include/nplbm.h).

Argument marshalling only: every step of the method runs in the library's
gfx950 kernels.  PyTorch provides the device memory (a uint8 tensor handed to
``nplbm_create``) and the stream (torch's current stream), so the library's
launches are ordered with the caller's torch work.

There is no CPU fallback: if the library is missing or no GPU is present the
calls fail loudly.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# NPLBM_LIB lets a developer point the binding at another build of the same
# library (A/B timing of kernel variants); the default is the in-tree build.
LIB_PATH = os.environ.get("NPLBM_LIB") or os.path.join(HERE, "libnplbm.so")

NPLBM_OK = 0
ERRORS = {-1: "EINVAL", -2: "ENOTSPD", -3: "ENOMEM", -4: "EDEVICE", -5: "ETOOBIG",
          -6: "ESTATE", -7: "ENOTFOUND"}
# nplbm_result keeps the ticket only while the request is unfinished
ERRORS_KEEP_TICKET = -6

# every symbol declared in include/nplbm.h
EXPORTS = [
    "nplbm_last_error", "nplbm_validate", "nplbm_footprint", "nplbm_create",
    "nplbm_set_fields", "nplbm_step", "nplbm_get_c", "nplbm_get_u", "nplbm_get_p",
    "nplbm_diagnostics", "nplbm_diagnostics_noalloc", "nplbm_laplace", "nplbm_laplace3", "nplbm_time", "nplbm_sync", "nplbm_destroy",
    "nplbm_state_bytes", "nplbm_get_state", "nplbm_set_state", "nplbm_device_copy",
    "nplbm_server_create", "nplbm_submit", "nplbm_server_pump", "nplbm_poll",
    "nplbm_result", "nplbm_server_stats", "nplbm_server_destroy",
]


class NplbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"nplbm error {ERRORS.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("wall_y", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("grad_scheme", ctypes.c_int32), ("force_form", ctypes.c_int32),
                ("sigma", ctypes.POINTER(ctypes.c_double)),
                ("rho", ctypes.POINTER(ctypes.c_double)),
                ("mu", ctypes.POINTER(ctypes.c_double)),
                ("mobility", ctypes.POINTER(ctypes.c_double)),
                ("tau_phi", ctypes.POINTER(ctypes.c_double)),
                ("interface_width", ctypes.c_double),
                ("gx", ctypes.c_double), ("gy", ctypes.c_double),
                ("gz", ctypes.c_double), ("nz", ctypes.c_int32), ("wall_z", ctypes.c_int32)]


_LIB = None


def lib():
    """Load libnplbm.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1904_12553_amd.build_lib`")
        # torch first: its HIP runtime is then the one the library binds to
        # (same soname), so streams and device memory handed over from torch
        # belong to the library's runtime.  Loaded the other way round, the
        # process holds two HIP runtimes and the library's may see no device.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        c_int, c_i32, c_i64, c_u64 = ctypes.c_int, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        vp, dp, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t
        PP = ctypes.POINTER(Params)
        sig = {
            "nplbm_last_error": ([], ctypes.c_char_p),
            "nplbm_validate": ([PP, dp, dp, dp], c_int),
            "nplbm_footprint": ([PP], sz),
            "nplbm_create": ([PP, vp, vp, sz, ctypes.POINTER(vp)], c_int),
            "nplbm_set_fields": ([vp, dp, dp], c_int),
            "nplbm_step": ([vp, c_i64], c_int),
            "nplbm_get_c": ([vp, dp], c_int),
            "nplbm_get_u": ([vp, dp], c_int),
            "nplbm_get_p": ([vp, dp], c_int),
            "nplbm_diagnostics": ([vp, dp, dp, ctypes.POINTER(c_i64)], c_int),
            "nplbm_diagnostics_noalloc": ([vp, vp], c_int),
            "nplbm_laplace3": ([vp] + [ctypes.c_double] * 5 + [dp], c_int),
            "nplbm_laplace": ([vp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, dp], c_int),
            "nplbm_time": ([vp], c_i64),
            "nplbm_sync": ([vp], c_int),
            "nplbm_destroy": ([vp], None),
            "nplbm_state_bytes": ([vp], sz),
            "nplbm_get_state": ([vp, vp, ctypes.POINTER(c_i64)], c_int),
            "nplbm_set_state": ([vp, vp, c_i64], c_int),
            "nplbm_device_copy": ([vp, vp, sz, vp], c_int),
            "nplbm_server_create": ([sz, c_i32, c_i32, vp, ctypes.POINTER(vp)], c_int),
            "nplbm_submit": ([vp, PP, dp, dp, c_i64, ctypes.POINTER(c_u64)], c_int),
            "nplbm_server_pump": ([vp, ctypes.POINTER(c_i32)], c_int),
            "nplbm_poll": ([vp, c_u64, ctypes.POINTER(c_i32)], c_int),
            "nplbm_result": ([vp, c_u64, dp, dp, dp, dp, dp], c_int),
            "nplbm_server_stats": ([vp, dp, dp, dp, dp, dp, ctypes.POINTER(c_i64)], c_int),
            "nplbm_server_destroy": ([vp], None),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _LIB = L
    return _LIB


def _check(rc: int):
    if rc != NPLBM_OK:
        raise NplbmError(rc, lib().nplbm_last_error().decode())


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(N, nx, ny, sigma, rho, mu, mobility=0.1, tau_phi=0.8, W=4.0, wall_y=False,
                gx=0.0, gy=0.0, precision=64, grad_scheme=0, force_form=0, nz=1, wall_z=False,
                gz=0.0):
    """Build a Params struct; returns (struct, keepalive arrays).  nz >= 4
    makes a 3-D (D3Q15) domain."""
    arr = lambda x, n: np.ascontiguousarray(np.broadcast_to(np.asarray(x, np.float64), (n,)))
    sig = np.ascontiguousarray(np.asarray(sigma, np.float64).reshape(N, N))
    keep = (sig, arr(rho, N), arr(mu, N), arr(mobility, N - 1), arr(tau_phi, N - 1))
    p = Params(N=N, nx=nx, ny=ny, wall_y=int(bool(wall_y)), precision=int(precision),
               grad_scheme=int(grad_scheme), force_form=int(force_form), sigma=_dp(keep[0]),
               rho=_dp(keep[1]),
               mu=_dp(keep[2]), mobility=_dp(keep[3]), tau_phi=_dp(keep[4]),
               interface_width=float(W), gx=float(gx), gy=float(gy), gz=float(gz),
               nz=int(nz), wall_z=int(bool(wall_z)))
    return p, keep


def validate(N, sigma, rho, mu=None, mobility=0.1, tau_phi=0.8, W=4.0, nx=8, ny=8,
             grad_scheme=0, force_form=0):
    """Host-only check of a parameter set; returns (lambda, beta2, K)."""
    mu = np.ones(N) if mu is None else mu
    p, keep = make_params(N, nx, ny, sigma, rho, mu, mobility, tau_phi, W,
                          grad_scheme=grad_scheme, force_form=force_form)
    lam = np.empty((N - 1) * (N - 1))
    b2, K = ctypes.c_double(), ctypes.c_double()
    _check(lib().nplbm_validate(ctypes.byref(p), _dp(lam), ctypes.byref(b2), ctypes.byref(K)))
    return lam.reshape(N - 1, N - 1), b2.value, K.value


def accepts(sigma, rho) -> bool:
    """True when the library accepts (sigma, rho): eq:N14 has an SPD solution."""
    try:
        validate(len(rho), sigma, rho)
    except NplbmError:
        return False
    return True


def footprint(**kw) -> int:
    p, keep = make_params(**kw)
    return int(lib().nplbm_footprint(ctypes.byref(p)))


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the nplbm library runs on the GPU only")
    return torch


class Domain:
    """One lattice domain on the GPU.

    Keyword arguments are those of ``make_params``.  Device memory is a
    torch uint8 tensor on ``device`` handed to the library.  All launches go
    to ``stream`` (a torch stream), by default a stream of the domain's own
    (default priority): step runs are replayed as HIP graphs, which the
    null stream (torch's default) cannot capture.
    """

    def __init__(self, device: str = "cuda:0", stream=None, **kw):
        torch = _torch()
        self.N, self.nx, self.ny = int(kw["N"]), int(kw["nx"]), int(kw["ny"])
        self.nz = int(kw.get("nz", 1))
        self.dim = 3 if self.nz > 1 else 2
        self.precision = int(kw.get("precision", 64))
        self._p, self._keep = make_params(**kw)
        L = lib()
        nbytes = int(L.nplbm_footprint(ctypes.byref(self._p)))
        if nbytes == 0:
            _check(L.nplbm_validate(ctypes.byref(self._p), None, None, None))
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
            self.mem = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            # the buffer is used on self.stream from here on
            torch.cuda.current_stream(self.device).synchronize()
            ptr = self.mem.data_ptr()
            aligned = (ptr + 255) & ~255
            h = ctypes.c_void_p()
            _check(L.nplbm_create(ctypes.byref(self._p), ctypes.c_void_p(self.stream.cuda_stream),
                                  ctypes.c_void_p(aligned), nbytes, ctypes.byref(h)))
        self._h = h
        self.footprint = nbytes

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().nplbm_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n(self):
        return self.nx * self.ny * max(self.nz, 1)

    @property
    def shape(self):
        """Shape of one field: (ny, nx) in 2-D, (nz, ny, nx) in 3-D."""
        return (self.nz, self.ny, self.nx) if self.dim == 3 else (self.ny, self.nx)

    @property
    def handle(self):
        return self._h

    def set_fields(self, c, u=None):
        c = np.ascontiguousarray(c, np.float64).reshape((self.N,) + self.shape)
        u = None if u is None else np.ascontiguousarray(u, np.float64).reshape(
            (self.dim,) + self.shape)
        _check(lib().nplbm_set_fields(self._h, _dp(c), _dp(u)))

    def step(self, n: int = 1):
        _check(lib().nplbm_step(self._h, int(n)))

    def sync(self):
        _check(lib().nplbm_sync(self._h))

    @property
    def time(self) -> int:
        return int(lib().nplbm_time(self._h))

    def get_c(self):
        out = np.empty((self.N,) + self.shape)
        _check(lib().nplbm_get_c(self._h, _dp(out)))
        return out

    def get_u(self):
        out = np.empty((self.dim,) + self.shape)
        _check(lib().nplbm_get_u(self._h, _dp(out)))
        return out

    def get_p(self):
        out = np.empty(self.shape)
        _check(lib().nplbm_get_p(self._h, _dp(out)))
        return out

    def macro(self):
        return self.get_c(), self.get_u(), self.get_p()

    def diagnostics(self):
        mass = np.empty(self.N)
        dev = ctypes.c_double()
        bad = ctypes.c_int64()
        _check(lib().nplbm_diagnostics(self._h, _dp(mass), ctypes.byref(dev), ctypes.byref(bad)))
        return mass, dev.value, bad.value

    def diagnostics_noalloc(self, out):
        """nplbm_diagnostics_noalloc into ``out``, a float64 device tensor of
        at least N + 2 elements (asynchronous on the domain's stream)."""
        torch = _torch()
        if out.dtype != torch.float64 or not out.is_cuda or out.numel() < self.N + 2 \
                or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 device tensor of N + 2 elements")
        _check(lib().nplbm_diagnostics_noalloc(self._h, ctypes.c_void_p(out.data_ptr())))

    def laplace(self, xc, yc, r_in, r_out, zc=None) -> float:
        """Laplace jump about (xc, yc) in 2-D, about (xc, yc, zc) in 3-D."""
        dp = ctypes.c_double()
        if self.dim == 3:
            _check(lib().nplbm_laplace3(self._h, float(xc), float(yc), float(zc), float(r_in),
                                        float(r_out), ctypes.byref(dp)))
        else:
            _check(lib().nplbm_laplace(self._h, float(xc), float(yc), float(r_in), float(r_out),
                                       ctypes.byref(dp)))
        return dp.value

    def get_state(self):
        nb = int(lib().nplbm_state_bytes(self._h))
        buf = np.empty(nb, np.uint8)
        t = ctypes.c_int64()
        _check(lib().nplbm_get_state(self._h, buf.ctypes.data_as(ctypes.c_void_p), ctypes.byref(t)))
        return buf, t.value

    def set_state(self, buf, t):
        buf = np.ascontiguousarray(buf, np.uint8)
        _check(lib().nplbm_set_state(self._h, buf.ctypes.data_as(ctypes.c_void_p), int(t)))


def device_copy(dst, src, nbytes: int, stream=None):
    """Plain copy kernel between two device tensors (asynchronous)."""
    torch = _torch()
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().nplbm_device_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                                   int(nbytes), ctypes.c_void_p(st.cuda_stream)))


class Server:
    """Continuous-batching server (see include/nplbm.h)."""

    def __init__(self, hbm_budget: int, max_slots: int = 256, quantum: int = 50, stream=None):
        torch = _torch()
        self.stream = stream if stream is not None else torch.cuda.Stream()
        h = ctypes.c_void_p()
        _check(lib().nplbm_server_create(int(hbm_budget), int(max_slots), int(quantum),
                                         ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self._shapes = {}

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().nplbm_server_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, c, u=None, nsteps=1000, **kw) -> int:
        p, keep = make_params(**kw)
        N, nx, ny = kw["N"], kw["nx"], kw["ny"]
        c = np.ascontiguousarray(c, np.float64).reshape(N, ny, nx)
        u = None if u is None else np.ascontiguousarray(u, np.float64).reshape(2, ny, nx)
        t = ctypes.c_uint64()
        _check(lib().nplbm_submit(self._h, ctypes.byref(p), _dp(c), _dp(u), int(nsteps),
                                  ctypes.byref(t)))
        self._shapes[t.value] = (N, ny, nx)
        return t.value

    def pump(self) -> int:
        a = ctypes.c_int32()
        _check(lib().nplbm_server_pump(self._h, ctypes.byref(a)))
        return a.value

    def poll(self, ticket: int) -> int:
        s = ctypes.c_int32()
        _check(lib().nplbm_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(s)))
        return s.value

    def result(self, ticket: int):
        """(c, u, p, admit_s, done_s) of a finished request.  A failed
        request raises its error (and is forgotten); a request still queued
        or resident raises NPLBM_ESTATE and keeps its ticket."""
        if ticket not in self._shapes:   # unknown here: the library says why
            _check(lib().nplbm_result(self._h, ctypes.c_uint64(ticket), None, None, None,
                                      None, None))
        N, ny, nx = self._shapes[ticket]
        c = np.empty((N, ny, nx))
        u = np.empty((2, ny, nx))
        p = np.empty((ny, nx))
        a, d = ctypes.c_double(), ctypes.c_double()
        rc = lib().nplbm_result(self._h, ctypes.c_uint64(ticket), _dp(c), _dp(u), _dp(p),
                                ctypes.byref(a), ctypes.byref(d))
        if rc != ERRORS_KEEP_TICKET:
            self._shapes.pop(ticket, None)
        _check(rc)
        return c, u, p, a.value, d.value

    def stats(self) -> dict:
        """Aggregate statistics of the server (include/nplbm.h)."""
        p50, p99, ml, nu, busy = (ctypes.c_double() for _ in range(5))
        done = ctypes.c_int64()
        _check(lib().nplbm_server_stats(self._h, ctypes.byref(p50), ctypes.byref(p99),
                                        ctypes.byref(ml), ctypes.byref(nu), ctypes.byref(busy),
                                        ctypes.byref(done)))
        return {"p50_s": p50.value, "p99_s": p99.value, "mlups": ml.value,
                "node_updates": nu.value, "busy_s": busy.value, "completed": done.value}
