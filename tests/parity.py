"""Parity helpers: compare HIP results with the oracle under the scaled
tolerance |gpu - oracle| <= tol * S, with S the oracle's FP64 magnitude bound
sum |c(t)| |x^a| of every entry (entries with S = 0 must be exactly zero).

Tolerances: 1e-12 (double), 1e-26 (double double), 1e-52 (quad double).
Expected margin from the arithmetic: each entry is a sum of at most a few
hundred products of <= 40 factors, each operation adding a relative error of
about u_L (2^-53, 2^-104, 2^-205), so |error| <~ 10^3 u_L S: 1e-13 S,
5e-29 S and 2e-59 S -- one to seven orders of magnitude below the bars.
"""
import numpy as np

from tests.exact import limb_sum_diff

TOL = {1: 1e-12, 2: 1e-26, 4: 1e-52}


def scaled_error(gpu, ora, scale):
    """max over entries of |gpu - ora| / S, with gpu/ora [..., 2, L] and S [...]."""
    d = np.abs(limb_sum_diff(gpu, ora)).max(axis=-1)       # [...] worst of re/im
    s = np.asarray(scale)
    zero = s == 0
    if np.any(zero):
        assert np.all(np.asarray(gpu)[zero] == 0), "entries with S = 0 must be exactly zero"
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(zero, 0.0, d / np.where(zero, 1.0, s))
    return float(np.max(r)) if r.size else 0.0
