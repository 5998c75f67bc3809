"""The allocation-free diagnostics entry point (nplbm_diagnostics_noalloc):
its reduction scratch is a static device array of the library, its output a
caller-owned device buffer.  Checked against nplbm_diagnostics on the same
state, bitwise (the same kernels over the same block count), on two calls
in a row, the second on a smaller domain (the static array then still holds
the first call's larger set of partial records)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _case(w, steps, precision):
    import torch

    import paper_1904_12553_amd as P
    d = P.Domain(precision=precision, **w.params())
    d.set_fields(w.c, w.u)
    d.step(steps)
    out = torch.full((w.N + 2,), float("nan"), dtype=torch.float64, device="cuda")
    d.diagnostics_noalloc(out)
    d.sync()
    got = out.cpu().numpy()
    mass, dev, bad = d.diagnostics()
    d.close()
    return got, np.concatenate([mass, [dev, float(bad)]])


def test_noalloc_diagnostics_equal_the_allocating_call():
    from oracle.accept import oracle_accepts
    print("case no-alloc diagnostics: 1024x768 N=5 fp32, then 100x60 N=3 fp64", flush=True)
    big = W.bands_and_droplets(1024, ndrop=16, accept=oracle_accepts)
    small = W.random_smooth(3, 100, 60, seed=5, wall_y=True, accept=oracle_accepts)
    for w, steps, prec in ((big, 30, 32), (small, 17, 64)):
        got, ref = _case(w, steps, prec)
        assert np.array_equal(got, ref), (w.N, w.nx, w.ny, got, ref)
        assert ref[w.N + 1] == 0.0 and ref[w.N] < 1e-5


def test_noalloc_diagnostics_reject_bad_arguments():
    import paper_1904_12553_amd as P
    from paper_1904_12553_amd import nplbm as nb
    w = W.static_droplet(64, 64, R=16)
    d = P.Domain(precision=64, **w.params())
    with pytest.raises(nb.NplbmError) as e:   # before set_fields
        import torch
        d.diagnostics_noalloc(torch.zeros(8, dtype=torch.float64, device="cuda"))
    assert e.value.code == -6
    rc = nb.lib().nplbm_diagnostics_noalloc(d.handle, None)
    assert rc == -1
    d.close()
