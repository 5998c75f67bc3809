"""The largest 2-D lattice the library accepts for its row addressing: a
row block of one state group (all its planes of one lattice row) just
below 2^31 bytes, so every 32-bit byte offset of the step kernel is near
its limit.  N = 3 in FP64: 18 CH planes x 14 900 000 columns x 8 bytes =
2.1456e9 bytes per row block (limit 2^31 = 2.1475e9); 4 rows with walls,
60 million nodes, 34 GB of device memory.

The initial fields repeat with period 100 in x, so after any number of
steps the state is the 100 x 4 run tiled 149 000 times; every node is
compared bitwise with that run (the arithmetic of a node depends only on
its neighbourhood, not on its address or strip)."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle.accept import oracle_accepts
from tests.gpu_util import gpu_domain

pytestmark = pytest.mark.gpu

REPEAT = 149_000  # 100 * REPEAT = 14 900 000 columns


def test_largest_row_block_is_translation_invariant():
    import paper_1904_12553_amd as P
    small = W.random_smooth(3, 100, 4, seed=77, wall_y=True, accept=oracle_accepts)
    big = dataclasses.replace(small, nx=100 * REPEAT, c=np.tile(small.c, (1, 1, REPEAT)),
                              u=np.tile(small.u, (1, 1, REPEAT)))
    # accepted, and the first row of 32-column lines past the limit is not
    first_bad = -(-(1 << 31) // (18 * 8 * 32)) * 32
    assert P.footprint(precision=64, **big.params()) > 0
    assert P.footprint(precision=64, **dict(big.params(), nx=first_bad - 32)) > 0
    assert P.footprint(precision=64, **dict(big.params(), nx=first_bad)) == 0
    print(f"case {big.nx}x{big.ny} N=3 fp64 walls steps=12", flush=True)
    d = gpu_domain(small)
    d.step(12)
    ref = d.macro()
    d.close()
    d = gpu_domain(big)
    d.step(12)
    out = d.macro()
    m, dev, bad = d.diagnostics()
    d.close()
    for a, b in zip(out, ref):
        a = a.reshape(a.shape[:-1] + (REPEAT, 100))
        assert (a == b[..., None, :]).all()
    assert bad == 0 and dev < 1e-12


def test_largest_3d_plane_is_translation_invariant():
    """D3Q15, N = 3 in FP32: one plane of the CH group is 30 planes x 1088
    rows x 16416 (padded) columns x 4 bytes = 2.1433e9 bytes, just below the
    2^31 bound of the 3-D kernel's 32-bit offsets; 6 planes with walls in z,
    107 million nodes, 53 GB.  Fields of period 64 x 16 in x and y: bitwise
    equal to the 64 x 16 x 6 run tiled."""
    import paper_1904_12553_amd as P
    rx, ry = 256, 68
    small = W.random_smooth3d(3, 64, 16, 6, seed=78, wall_z=True, accept=oracle_accepts)
    big = dataclasses.replace(small, nx=64 * rx, ny=16 * ry,
                              c=np.tile(small.c, (1, 1, ry, rx)), u=np.tile(small.u, (1, 1, ry, rx)))
    assert P.footprint(precision=32, **big.params()) > 0
    print(f"case {big.nx}x{big.ny}x{big.nz} N=3 fp32 walls steps=10", flush=True)
    d = gpu_domain(small, precision=32)
    d.step(10)
    ref = d.macro()
    d.close()
    d = gpu_domain(big, precision=32)
    d.step(10)
    out = d.macro()
    d.close()
    for a, b in zip(out, ref):
        a = a.reshape(a.shape[:-2] + (ry, 16, rx, 64))
        assert (a == b.reshape(b.shape[:-2] + (1, 16, 1, 64))).all()
