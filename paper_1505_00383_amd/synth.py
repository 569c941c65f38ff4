"""Seeded synthetic workloads: polynomial systems, points and path subsets.

This module draws inputs only.  It holds none of the method's arithmetic (no
evaluation, no differentiation, no solving) and imports neither the oracle nor
the HIP library, so both sides can be fed the very same arrays.

A system is stored in a compressed sparse layout shared by every consumer:

* ``eq_term_off[n_eq+1]``   -- terms of equation i are ``eq_term_off[i]:eq_term_off[i+1]``
* ``term_fac_off[T+1]``     -- factors of term s are ``term_fac_off[s]:term_fac_off[s+1]``
  (k = count; k = 0 is a constant term)
* ``fac_var``, ``fac_exp``  -- variable index (strictly increasing inside a term) and
  exponent (>= 1) of each factor
* ``coef[T, 2]``            -- complex coefficient (re, im) in FP64

Coefficients and gamma are points on the unit circle, (cos th, sin th) with
th ~ U[0, 2 pi): the paper draws its constant gamma at random (Section 1, Eq. (1)),
and its benchmark systems are not available, so random unit-modulus
coefficients stand in for them.  The system is *defined* by those FP64 values;
higher limbs of coefficients are zero.

Random generator: numpy PCG64 seeded with 20150501 + workload index, draws taken
in a fixed order (monomial sets and angles per equation, then gamma, then the
points / t values or the path subset).
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 20150501


@dataclass
class System:
    n_eq: int
    n_var: int
    eq_term_off: np.ndarray
    term_fac_off: np.ndarray
    fac_var: np.ndarray
    fac_exp: np.ndarray
    coef: np.ndarray  # [T, 2] float64
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_terms(self) -> int:
        return int(self.eq_term_off[-1])

    def degrees(self) -> np.ndarray:
        """Total degree of every equation (max over its terms of the exponent sum)."""
        d = np.zeros(self.n_eq, dtype=np.int32)
        for i in range(self.n_eq):
            best = 0
            for s in range(self.eq_term_off[i], self.eq_term_off[i + 1]):
                a, b = self.term_fac_off[s], self.term_fac_off[s + 1]
                best = max(best, int(self.fac_exp[a:b].sum()))
            d[i] = best
        return d

    def terms(self, i: int):
        """Yield (coef complex, [(var, exp), ...]) for equation i."""
        for s in range(self.eq_term_off[i], self.eq_term_off[i + 1]):
            a, b = self.term_fac_off[s], self.term_fac_off[s + 1]
            yield (complex(self.coef[s, 0], self.coef[s, 1]),
                   [(int(v), int(e)) for v, e in zip(self.fac_var[a:b], self.fac_exp[a:b])])


def system_from_terms(n_var: int, eqs, name: str = "", meta=None) -> System:
    """Build a System from ``eqs[i] = [(coef, {var: exp}), ...]``."""
    eq_off = [0]
    tf_off = [0]
    fv, fe, cf = [], [], []
    for eq in eqs:
        for c, mono in eq:
            items = sorted((int(v), int(e)) for v, e in dict(mono).items() if int(e) > 0)
            for v, e in items:
                if not (0 <= v < n_var):
                    raise ValueError("variable index out of range")
                fv.append(v)
                fe.append(e)
            tf_off.append(len(fv))
            c = complex(c)
            cf.append((c.real, c.imag))
        eq_off.append(len(cf))
    return System(
        n_eq=len(eqs), n_var=n_var,
        eq_term_off=np.asarray(eq_off, dtype=np.int32),
        term_fac_off=np.asarray(tf_off, dtype=np.int32),
        fac_var=np.asarray(fv, dtype=np.int32),
        fac_exp=np.asarray(fe, dtype=np.int32),
        coef=np.asarray(cf, dtype=np.float64).reshape(-1, 2),
        name=name, meta=dict(meta or {}))


def unit_complex(rng: np.random.Generator) -> complex:
    th = rng.uniform(0.0, 2.0 * math.pi)
    return complex(math.cos(th), math.sin(th))


def monomials_upto(nvars_list, deg: int):
    """All exponent dicts over the given variables with total degree <= deg (includes 1)."""
    out = []
    nv = len(nvars_list)
    for total in range(deg + 1):
        for combo in itertools.combinations_with_replacement(range(nv), total):
            m = {}
            for c in combo:
                v = nvars_list[c]
                m[v] = m.get(v, 0) + 1
            out.append(m)
    return out


def _key(m):
    return tuple(sorted(m.items()))


def _equation_with_anchor(rng, variables, i, d, n_terms):
    """Equation i: x_i^d, the constant 1, and n_terms-2 distinct other monomials of
    degree <= d over ``variables`` drawn without replacement, each with a random
    unit coefficient.  Having x_i^d - 1 inside the coefficient family keeps the
    family generic for total-degree homotopies (x = 0 is not forced to be a root)."""
    anchor = {i: d}
    const = {}
    pool = [m for m in monomials_upto(variables, d)
            if _key(m) != _key(anchor) and _key(m) != _key(const)]
    if n_terms - 2 > len(pool):
        raise ValueError("not enough monomials for the requested term count")
    pick = rng.choice(len(pool), size=n_terms - 2, replace=False)
    monos = [anchor, const] + [pool[int(p)] for p in pick]
    return [(unit_complex(rng), m) for m in monos]


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def tracking_small(seed: int = SEED_BASE + 0):
    """n = 3 equations in 3 unknowns, 4 monomials each (x_i^2, 1, two others of
    degree <= 2); start system x_i^2 - 1, 8 paths, gamma a random unit complex."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = 3
    eqs = [_equation_with_anchor(rng, list(range(n)), i, 2, 4) for i in range(n)]
    gamma = unit_complex(rng)
    return system_from_terms(n, eqs, name="track-n3-d2", meta={"gamma": gamma, "paths": 8})


def eval_dense(seed: int = SEED_BASE + 1, n: int = 32, terms_per_eq: int = 64, k: int = 8,
               max_exp: int = 3):
    """Evaluation workload: n equations and unknowns, ``terms_per_eq`` monomials per
    equation, each over k distinct variables chosen uniformly, exponents uniform in
    1..max_exp, unit-modulus coefficients."""
    rng = np.random.Generator(np.random.PCG64(seed))
    eqs = []
    for i in range(n):
        eq = []
        for _ in range(terms_per_eq):
            vars_ = np.sort(rng.choice(n, size=k, replace=False))
            exps = rng.integers(1, max_exp + 1, size=k)
            eq.append((unit_complex(rng), {int(v): int(e) for v, e in zip(vars_, exps)}))
        eqs.append(eq)
    gamma = unit_complex(rng)
    sysm = system_from_terms(n, eqs, name=f"eval-n{n}-T{terms_per_eq}-k{k}",
                             meta={"gamma": gamma})
    sysm.meta["rng_state"] = rng.bit_generator.state
    return sysm


def torus_points(sysm: System, npts: int, limbs: int, rng: np.random.Generator | None = None):
    """Points on the unit torus (phi ~ U[0, 2 pi) per coordinate) and t ~ U[0, 1).

    Returns (x[npts, nvar, 2, limbs], t[npts]).  For limbs > 1 every lower limb is
    a random fraction of half an ulp of the limb above it, so the full width of
    the multi-limb arithmetic is exercised.  Continues the workload's generator
    (drawn after gamma) unless ``rng`` is given."""
    if rng is None:
        rng = np.random.Generator(np.random.PCG64(0))
        rng.bit_generator.state = sysm.meta["rng_state"]
    phi = rng.uniform(0.0, 2.0 * math.pi, size=(npts, sysm.n_var))
    x = np.zeros((npts, sysm.n_var, 2, limbs), dtype=np.float64)
    x[:, :, 0, 0] = np.cos(phi)
    x[:, :, 1, 0] = np.sin(phi)
    for l in range(1, limbs):
        u = rng.uniform(-0.5, 0.5, size=(npts, sysm.n_var, 2))
        x[:, :, :, l] = u * np.spacing(np.abs(x[:, :, :, l - 1]))
    t = rng.uniform(0.0, 1.0, size=npts)
    return x, t


def random_points(n_var: int, npts: int, limbs: int, rng: np.random.Generator, scale: float = 1.0):
    """Complex Gaussian points (any modulus) with random lower limbs."""
    x = np.zeros((npts, n_var, 2, limbs), dtype=np.float64)
    x[:, :, :, 0] = rng.normal(size=(npts, n_var, 2)) * scale
    for l in range(1, limbs):
        u = rng.uniform(-0.5, 0.5, size=(npts, n_var, 2))
        x[:, :, :, l] = u * np.spacing(np.abs(x[:, :, :, l - 1]))
    return x


def tracking_cubic(seed: int = SEED_BASE + 2):
    """n = 8, every equation of degree exactly 3 with 20 monomials (x_i^3, 1 and 18
    others of degree <= 3 in all 8 unknowns); start x_i^3 - 1, 3^8 = 6561 paths."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = 8
    eqs = [_equation_with_anchor(rng, list(range(n)), i, 3, 20) for i in range(n)]
    gamma = unit_complex(rng)
    return system_from_terms(n, eqs, name="track-n8-d3", meta={"gamma": gamma, "paths": 3 ** 8})


def tracking_quadratic16(seed: int = SEED_BASE + 3):
    """n = 16, degree 2: equation i draws 16 monomials over x_i plus 5 other seeded
    unknowns (x_i^2, 1 and 14 others of degree <= 2 on those 6); start x_i^2 - 1,
    2^16 = 65536 paths."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = 16
    eqs = []
    for i in range(n):
        others = rng.choice([v for v in range(n) if v != i], size=5, replace=False)
        variables = sorted([i] + [int(v) for v in others])
        eqs.append(_equation_with_anchor(rng, variables, i, 2, 16))
    gamma = unit_complex(rng)
    return system_from_terms(n, eqs, name="track-n16-d2", meta={"gamma": gamma, "paths": 2 ** 16})


def batch_heterogeneous(seed: int = SEED_BASE + 4, nsys: int = 64, target_paths: int = 200_000,
                        n_range=(4, 16), terms_range=(8, 32)):
    """``nsys`` random systems, n ~ U{4..16}, per-equation degree ~ U{2,3}, terms per
    equation ~ U{8..32} (each includes x_i^{d_i} and 1).  Returns (systems, gammas,
    path lists).  Paths: every multi-index of the total-degree start system when its
    Bezout number B_s is at most a cap c, else a seeded random subset of c
    multi-indices; c is the smallest integer with sum_s min(B_s, c) >= target_paths."""
    rng = np.random.Generator(np.random.PCG64(seed))
    systems, gammas = [], []
    for s in range(nsys):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        degs = rng.integers(2, 4, size=n)
        eqs = []
        for i in range(n):
            d = int(degs[i])
            n_pool = len(monomials_upto(list(range(n)), d)) - 2
            nt = int(rng.integers(terms_range[0], terms_range[1] + 1))
            nt = min(nt, n_pool + 2)
            eqs.append(_equation_with_anchor(rng, list(range(n)), i, d, nt))
        systems.append(system_from_terms(n, eqs, name=f"batch-{s}-n{n}"))
        gammas.append(unit_complex(rng))
    bez = [int(np.prod(sy.degrees().astype(np.int64))) for sy in systems]
    lo, hi = 1, max(bez)
    while lo < hi:
        mid = (lo + hi) // 2
        if sum(min(b, mid) for b in bez) >= target_paths:
            hi = mid
        else:
            lo = mid + 1
    cap = lo
    paths = []
    for b in bez:
        if b <= cap:
            paths.append(np.arange(b, dtype=np.int64))
        else:
            paths.append(np.sort(rng.choice(b, size=cap, replace=False)).astype(np.int64))
    return systems, gammas, paths, cap


# ---------------------------------------------------------------------------
# Stand-ins shaped like the paper's three benchmark systems (Section 4 lists
# their dimensions, monomial counts and degrees).  Only the shape is taken:
# the supports are drawn at random (multilinear monomials over random
# variable subsets) and every coefficient is a random unit complex number, so
# none of the actual systems is reproduced.
# ---------------------------------------------------------------------------

def _subsets(n, sizes):
    return [c for d in sizes for c in itertools.combinations(range(n), d)]


def _multilinear_equation(rng, n, n_terms, sizes, must=()):
    """``n_terms`` distinct multilinear monomials over n unknowns, drawn without
    replacement from the variable subsets whose size is in ``sizes``; one of
    each size in ``must`` first."""
    pool = _subsets(n, sizes)
    picked = []
    for d in must:
        cands = [i for i, c in enumerate(pool) if len(c) == d and i not in picked]
        picked.append(cands[int(rng.integers(0, len(cands)))])
    rest = [i for i in range(len(pool)) if i not in set(picked)]
    picked += [rest[int(j)] for j in rng.choice(len(rest), size=n_terms - len(picked), replace=False)]
    return [(unit_complex(rng), {v: 1 for v in pool[i]}) for i in picked]


def shaped_cyclic10(seed: int = SEED_BASE + 10):
    """n = 10; equation k (k = 1..9) has 10 monomials of degree k, the last
    equation two terms (a monomial in all 10 unknowns and a constant): 92
    monomials, the shape of the cyclic 10-roots system."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = 10
    eqs = [_multilinear_equation(rng, n, 10, [k]) for k in range(1, n)]
    eqs.append([(unit_complex(rng), {v: 1 for v in range(n)}), (unit_complex(rng), {})])
    gamma = unit_complex(rng)
    return system_from_terms(n, eqs, name="shaped-cyclic10", meta={"gamma": gamma, "paths": 34940})


def shaped_nash8(seed: int = SEED_BASE + 11):
    """n = 8; every equation has 130 multilinear monomials of degrees 1..7
    (every degree present; 1040 monomials in all), the shape of the 8-player
    Nash equilibrium system."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = 8
    eqs = [_multilinear_equation(rng, n, 130, range(1, 8), must=range(1, 8)) for _ in range(n)]
    gamma = unit_complex(rng)
    return system_from_terms(n, eqs, name="shaped-nash8", meta={"gamma": gamma, "paths": 14833})


def shaped_pieri44(seed: int = SEED_BASE + 12):
    """n = 16; every equation has 246 multilinear monomials of degree at most
    4, at least one of degree 4 (3936 in all), the shape of the Pieri
    hypersurface system with four-planes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = 16
    eqs = [_multilinear_equation(rng, n, 246, range(1, 5), must=(4,)) for _ in range(n)]
    gamma = unit_complex(rng)
    return system_from_terms(n, eqs, name="shaped-pieri44", meta={"gamma": gamma, "paths": 24024})


SHAPED = {"cyclic10": shaped_cyclic10, "nash8": shaped_nash8, "pieri44": shaped_pieri44}


def gamma_of(sysm: System) -> complex:
    return complex(sysm.meta["gamma"])
