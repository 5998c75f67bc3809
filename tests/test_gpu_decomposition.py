"""The result of a step does not depend on how the launch cuts the lattice
into strips (2-D) or tiles (D3Q15): every node's arithmetic is the same, so
c, u and p after any number of steps must be bitwise identical across strip
widths, strip heights (down to 2 rows, with strips starting next to walls
and ramps full of ghost rows) and workgroup counts, in both precisions and
all three schemes.  This needs no oracle, so it runs at sizes where every
strip shape occurs."""
import os

import numpy as np
import pytest

import workloads as W
from oracle.accept import oracle_accepts
from tests.gpu_util import gpu_domain

pytestmark = pytest.mark.gpu

DECOMP_2D = [
    {},
    {"NPLBM_MIN_STRIP_H": "2", "NPLBM_TARGET_BLOCKS": "4096"},
    {"NPLBM_MIN_STRIP_H": "6", "NPLBM_TARGET_BLOCKS": "300"},
    {"NPLBM_MIN_STRIP_H": "400"},
    {"NPLBM_TX": "32", "NPLBM_MIN_STRIP_H": "10"},
]
KEYS = ("NPLBM_MIN_STRIP_H", "NPLBM_TARGET_BLOCKS", "NPLBM_TX", "NPLBM_TY3")


def _run(w, env, steps, **kw):
    saved = {k: os.environ.pop(k, None) for k in KEYS}
    os.environ.update(env)
    try:
        d = gpu_domain(w, **kw)
        d.step(steps)
        out = np.concatenate([np.ravel(a) for a in d.macro()])
        d.close()
    finally:
        for k in KEYS:
            os.environ.pop(k, None)
            if saved[k] is not None:
                os.environ[k] = saved[k]
    return out


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("scheme", ["central", "mixed", "remark1"])
@pytest.mark.parametrize("wall", [True, False])
def test_2d_state_independent_of_strips(precision, scheme, wall):
    over = {"central": {}, "mixed": {"grad_scheme": 1}, "remark1": {"force_form": 1}}[scheme]
    w = W.random_smooth(4, 230, 97, seed=31 + wall, wall_y=wall, accept=oracle_accepts)
    print(f"case 230x97 N=4 {scheme} wall={wall} fp{precision} steps=30", flush=True)
    ref = _run(w, DECOMP_2D[0], 30, precision=precision, **over)
    for env in DECOMP_2D[1:]:
        st = _run(w, env, 30, precision=precision, **over)
        assert np.array_equal(st, ref), env


@pytest.mark.parametrize("precision", [64, 32])
@pytest.mark.parametrize("wall", [True, False])
def test_3d_state_independent_of_tiles(precision, wall):
    w = W.random_smooth3d(3, 70, 21, 33, seed=41 + wall, wall_z=wall, accept=oracle_accepts)
    print(f"case 70x21x33 N=3 wall={wall} fp{precision} steps=20", flush=True)
    ref = _run(w, {}, 20, precision=precision)
    for env in ({"NPLBM_TY3": "4" if precision == 64 else "8"}, {"NPLBM_TARGET_BLOCKS": "8"},
                {"NPLBM_TARGET_BLOCKS": "100000"}):
        st = _run(w, env, 20, precision=precision)
        assert np.array_equal(st, ref), env
