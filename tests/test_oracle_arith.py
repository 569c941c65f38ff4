"""Pins of the oracle's multi-limb arithmetic against exact rational arithmetic.

The oracle forms every result exactly (as an expansion) and cuts it to L limbs,
so each result must lie within 2^(1-52L) of the exact rational value, relative
to the result (measured worst case is below 2^(-1-52L)).  Division and square root are Newton
iterations; their bound is checked against the exact quotient / a squared
check.  Operands: random, cancelling, with spread exponents and signed zeros.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from tests.exact import fr, frc, limbs_of

LIMBS = [1, 2, 4]


def _rand_mp(rng, L, spread=True):
    e = int(rng.integers(-30, 30)) if spread else 0
    v = np.zeros(L)
    v[0] = rng.normal() * 2.0 ** e
    for l in range(1, L):
        v[l] = rng.uniform(-0.5, 0.5) * np.spacing(abs(v[l - 1]))
    return v


def _rel_ok(got: Fraction, exact: Fraction, L: int, slack: int = 1) -> bool:
    if exact == 0:
        return got == 0
    return abs(got - exact) <= abs(exact) * Fraction(2) ** (slack - 52 * L)


@pytest.mark.parametrize("L", LIMBS)
def test_add_sub_mul_exact_bound(L):
    rng = np.random.default_rng(1)
    for _ in range(300):
        a, b = _rand_mp(rng, L), _rand_mp(rng, L)
        A, B = fr(a), fr(b)
        assert _rel_ok(fr(oracle.mp_op(L, oracle.MP_ADD, a, b)), A + B, L)
        assert _rel_ok(fr(oracle.mp_op(L, oracle.MP_SUB, a, b)), A - B, L)
        assert _rel_ok(fr(oracle.mp_op(L, oracle.MP_MUL, a, b)), A * B, L)


@pytest.mark.parametrize("L", LIMBS)
def test_cancellation_and_identities(L):
    rng = np.random.default_rng(2)
    for _ in range(200):
        a = _rand_mp(rng, L)
        # a + (-a) == 0 exactly, a * 1 == a exactly
        assert fr(oracle.mp_op(L, oracle.MP_ADD, a, -a)) == 0
        assert fr(oracle.mp_op(L, oracle.MP_MUL, a, np.eye(1, L)[0])) == fr(a)
        # near-cancellation: b = a + tiny
        b = a.copy()
        b[-1] += np.spacing(abs(a[-1])) * 3 if a[-1] != 0 else 1e-300
        exact = fr(a) - fr(b)
        assert _rel_ok(fr(oracle.mp_op(L, oracle.MP_SUB, a, b)), exact, L)
    # signed zeros
    z = np.zeros(L)
    nz = -np.zeros(L)
    assert fr(oracle.mp_op(L, oracle.MP_ADD, z, nz)) == 0
    assert fr(oracle.mp_op(L, oracle.MP_MUL, nz, np.eye(1, L)[0])) == 0


@pytest.mark.parametrize("L", LIMBS)
def test_div_sqrt(L):
    rng = np.random.default_rng(3)
    for _ in range(150):
        a, b = _rand_mp(rng, L), _rand_mp(rng, L)
        q = fr(oracle.mp_op(L, oracle.MP_DIV, a, b))
        assert _rel_ok(q, fr(a) / fr(b), L, slack=4)
        pa = a if a[0] > 0 else -a  # positive operand
        s = fr(oracle.mp_op(L, oracle.MP_SQRT, pa))
        # |s^2 - a| <= 2 * rel * a  <=> relative error of s about rel
        assert abs(s * s - fr(pa)) <= fr(pa) * Fraction(2) ** (5 - 52 * L)


@pytest.mark.parametrize("L", LIMBS)
def test_sqrt3_squared(L):
    s = fr(oracle.mp_op(L, oracle.MP_SQRT, np.eye(1, L)[0] * 3.0))
    assert abs(s * s - 3) <= 3 * Fraction(2) ** (3 - 52 * L)


@pytest.mark.parametrize("L", LIMBS)
def test_complex_ops_componentwise(L):
    rng = np.random.default_rng(4)
    for _ in range(200):
        a = np.stack([_rand_mp(rng, L, False), _rand_mp(rng, L, False)])
        b = np.stack([_rand_mp(rng, L, False), _rand_mp(rng, L, False)])
        ar, ai = frc(a)
        br, bi = frc(b)
        pr, pi = frc(oracle.cx_op(L, oracle.CX_MUL, a, b))
        assert _rel_ok(pr, ar * br - ai * bi, L)
        assert _rel_ok(pi, ar * bi + ai * br, L)
        cr, ci = frc(oracle.cx_op(L, oracle.CX_CMUL, a, b))
        assert _rel_ok(cr, ar * br + ai * bi, L)
        assert _rel_ok(ci, ar * bi - ai * br, L)
        sr, si = frc(oracle.cx_op(L, oracle.CX_ADD, a, b))
        assert _rel_ok(sr, ar + br, L) and _rel_ok(si, ai + bi, L)


def test_limbs_are_nonoverlapping():
    rng = np.random.default_rng(5)
    for L in (2, 4):
        for _ in range(100):
            a, b = _rand_mp(rng, L), _rand_mp(rng, L)
            r = oracle.mp_op(L, oracle.MP_MUL, a, b)
            for l in range(1, L):
                assert abs(r[l]) <= np.spacing(abs(r[l - 1])) or r[l] == 0


def test_limbs_of_roundtrip():
    q = Fraction(1, 3)
    for L in (1, 2, 4):
        v = limbs_of(q, L)
        assert abs(fr(v) - q) <= q * Fraction(2) ** (-52 * L)
