"""Helpers for the GPU tests: run the same seeded workload through the FP64
oracle and through the HIP library (via the C ABI binding)."""
import numpy as np

from oracle import OracleSim


def oracle_run(w, steps, **over):
    kw = w.params()
    kw.update(over)
    o = OracleSim(**kw)
    o.init(w.c, w.u)
    o.step(steps)
    return o


def gpu_domain(w, precision=64, **over):
    import paper_1904_12553_amd as P
    kw = w.params()
    kw.update(over)
    d = P.Domain(precision=precision, **kw)
    d.set_fields(w.c, w.u)
    return d


def maxabs(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))
