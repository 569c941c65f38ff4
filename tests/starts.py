"""Explicit start systems with closed-form roots, for tests of Eq. (1) with a
start system g other than the total-degree one.

g_i = a_i x_i^{d_i} - b_i with random complex a_i, b_i; its roots are
x_i = (b_i / a_i)^{1/d_i} omega^k, computed here with mpmath at 80 digits and
cut greedily into L limbs.  Test-side only: no part of the method is here.
"""
import numpy as np

from paper_1505_00383_amd import synth


def diagonal_start(rng, deg):
    """(system g, a, b) for g_i = a_i x_i^{d_i} - b_i."""
    a = [synth.unit_complex(rng) * (0.5 + rng.uniform()) for _ in deg]
    b = [synth.unit_complex(rng) * (0.5 + rng.uniform()) for _ in deg]
    g = synth.system_from_terms(len(deg), [[(a[i], {i: int(d)}), (-b[i], {})]
                                           for i, d in enumerate(deg)])
    return g, a, b


def diagonal_roots(a, b, deg, L, paths):
    """Roots of g for the listed multi-index numbers (little-endian mixed
    radix over deg) as [len(paths), n, 2, L] limb arrays."""
    import mpmath
    mpmath.mp.dps = 80
    X = np.zeros((len(paths), len(deg), 2, L))
    for q, p in enumerate(paths):
        rem = int(p)
        for i, d in enumerate(deg):
            k = rem % int(d)
            rem //= int(d)
            z = mpmath.root(mpmath.mpc(b[i].real, b[i].imag) / mpmath.mpc(a[i].real, a[i].imag),
                            int(d), k)
            for c, part in enumerate((z.real, z.imag)):
                r = part
                for l in range(L):
                    v = float(r)
                    X[q, i, c, l] = v
                    r -= mpmath.mpf(v)
    return X
