"""The x-halo of the central-scheme step kernel, where each lane of a row owns
an interior column and the phi of the four halo columns is pulled one lane
per (halo node, direction) (central scheme: FP32 for N <= 5, FP64 for
N <= 3; mixed and Remark 1 schemes: FP32 for N <= 5).

- FP64 against the oracle (1e-10 max-abs on c, u, p) on lattices narrower
  than the halo itself (nx = 4, 5: the halo columns wrap onto the strip's
  own columns), a one-column strip next to a full one (nx = 33 cut into
  strips of 32 and 1 columns), and with walls, where the halo lanes of
  the rows next to a wall take the bounce-back sources;
- FP32 and FP64 states bitwise identical across strip widths (256, 32, 8
  columns: every strip edge moves), so a halo phi equals, bit for bit, the
  phi the neighbouring strip computes for that node.
"""
import os

import numpy as np
import pytest

import workloads as W
from oracle.accept import oracle_accepts
from tests.gpu_util import gpu_domain, maxabs, oracle_run

pytestmark = pytest.mark.gpu
TOL = 1e-10
KEYS = ("NPLBM_TX",)


def _state(w, precision, steps, env, **over):
    saved = {k: os.environ.pop(k, None) for k in KEYS}
    os.environ.update(env)
    try:
        d = gpu_domain(w, precision=precision, **over)
        d.step(steps)
        out = [np.asarray(a) for a in d.macro()]
        d.close()
    finally:
        for k in KEYS:
            os.environ.pop(k, None)
            if saved[k] is not None:
                os.environ[k] = saved[k]
    return out


@pytest.mark.parametrize("N,nx,ny,wall,tx", [
    (3, 4, 9, False, None),
    (2, 5, 12, True, None),
    (3, 33, 6, True, "32"),
    (3, 33, 7, False, "32"),
    (2, 70, 10, True, "8"),
])
def test_halo_lanes_fp64_against_oracle(N, nx, ny, wall, tx):
    w = W.random_smooth(N, nx, ny, seed=9100 + nx + ny, wall_y=wall, accept=oracle_accepts)
    steps = 20
    print(f"case halo N={N} {nx}x{ny} wall={wall} tx={tx} fp64 steps={steps}", flush=True)
    o = oracle_run(w, steps)
    got = _state(w, 64, steps, {"NPLBM_TX": tx} if tx else {})
    err = [maxabs(a, b) for a, b in zip(got, o.macro())]
    assert max(err) < TOL, err


@pytest.mark.parametrize("precision,N,scheme", [(32, 2, "central"), (32, 3, "central"),
                                                (32, 5, "central"), (64, 2, "central"),
                                                (64, 3, "central"), (32, 3, "mixed"),
                                                (32, 5, "mixed"), (32, 3, "remark1"),
                                                (32, 5, "remark1")])
@pytest.mark.parametrize("wall", [False, True])
def test_halo_lanes_bitwise_across_strip_widths(precision, N, scheme, wall):
    w = W.random_smooth(N, 300, 23, seed=9200 + N + 10 * wall, wall_y=wall, accept=oracle_accepts)
    over = {"mixed": {"grad_scheme": 1}, "remark1": {"force_form": 1}}.get(scheme, {})
    print(f"case halo bitwise N={N} {scheme} 300x23 wall={wall} fp{precision} steps=30", flush=True)
    ref = _state(w, precision, 30, {}, **over)
    for tx in ("32", "8"):
        got = _state(w, precision, 30, {"NPLBM_TX": tx}, **over)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), tx


@pytest.mark.parametrize("scheme", ["mixed", "remark1"])
@pytest.mark.parametrize("N,nx,ny,wall", [(3, 5, 12, True), (4, 70, 9, False), (5, 33, 8, True)])
def test_two_hop_halo_lanes_fp32_against_fp64(N, nx, ny, wall, scheme):
    """The two-hop schemes' rows of interior lanes (FP32) against their FP64
    rows, which hold their halo, after 200 steps (FP32 state, FP64 NS
    arithmetic: agreement to 1e-5 on c), with strips of 32 columns so that
    the 3-column halo (and, for Remark 1, the previous u of the columns
    beside the interior) crosses strip edges."""
    over = {"mixed": {"grad_scheme": 1}, "remark1": {"force_form": 1}}[scheme]
    w = W.random_smooth(N, nx, ny, seed=9300 + nx, wall_y=wall, accept=oracle_accepts)
    print(f"case {scheme} halo N={N} {nx}x{ny} wall={wall} fp32 vs fp64 steps=200", flush=True)
    c32 = _state(w, 32, 200, {"NPLBM_TX": "32"}, **over)[0]
    c64 = _state(w, 64, 200, {}, **over)[0]
    assert maxabs(c32, c64) < 1e-5
