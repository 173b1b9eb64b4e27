"""Shared measure of agreement between a GPU result and the oracle.

relerr() is the larger of the normwise relative error ||x - ref||_2 / ||ref||_2
and the element-wise one max_i |x_i - ref_i| / ||ref||_inf, so a bound on it
also bounds every single component (a wrong small entry cannot hide under a
normwise bound).  NaN anywhere makes it NaN, which fails every `<=` test.
"""
import numpy as np


def relerr(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = x - ref
    nrm = float(np.linalg.norm(d) / max(np.linalg.norm(ref), 1e-300))
    elt = float(np.max(np.abs(d)) / max(np.max(np.abs(ref)), 1e-300)) if d.size else 0.0
    if np.isnan(nrm) or np.isnan(elt):
        return float("nan")
    return max(nrm, elt)
