"""Exact and high-precision helpers for the pins (test-side only).

Nothing here implements the method: these turn limb arrays into exact
rationals (``fractions.Fraction``) or mpmath numbers so that results of the
oracle and of the HIP path can be compared against exact mathematics.
"""
from fractions import Fraction

import numpy as np


def fr(limbs) -> Fraction:
    """Exact value of a multi-limb real (sum of its doubles)."""
    return sum((Fraction(float(v)) for v in np.ravel(limbs)), Fraction(0))


def frc(cl):
    """Exact value of a multi-limb complex stored as [2][L]."""
    cl = np.asarray(cl)
    return (fr(cl[0]), fr(cl[1]))


def limbs_of(q: Fraction, L: int) -> np.ndarray:
    """Greedy nearest-double limbs of an exact rational (test input maker)."""
    out = np.zeros(L)
    r = q
    for l in range(L):
        d = float(r)
        out[l] = d
        r -= Fraction(d)
    return out


def limb_sum_diff(a, b):
    """(sum of limbs of a) - (sum of limbs of b), elementwise over leading axes,
    accurate to a few ulps of the difference.  a, b: [..., L]."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    terms = np.concatenate([a, -b], axis=-1)
    # cascaded error-free summation (vectorised TwoSum passes) until stable
    for _ in range(terms.shape[-1] + 2):
        s = terms[..., 0].copy()
        errs = []
        for k in range(1, terms.shape[-1]):
            x = terms[..., k]
            t = s + x
            bv = t - s
            e = (s - (t - bv)) + (x - bv)
            s = t
            errs.append(e)
        terms = np.stack(errs + [s], axis=-1)
    return terms.sum(axis=-1)
