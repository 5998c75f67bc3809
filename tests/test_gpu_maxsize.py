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
