"""Pins of the oracle's evaluation of H(x,t) = gamma(1-t) g(x) + t f(x) and dH/dx.

Independent references:
* exact rational evaluation with sympy, derivatives by ``sympy.diff`` (not by
  the oracle's symbolic rule), on tiny systems including terms with k = 0, 1, 2,
  and 3 variables;
* central finite differences of the oracle's own H in quad double;
* Euler's identity for homogeneous equations, sum_j x_j dF_i/dx_j = d_i F_i;
* t = 1 gives f, t = 0 gives gamma * g; g vanishes at roots of unity.
"""
from fractions import Fraction

import numpy as np
import pytest
import sympy as sp

import oracle
from paper_1505_00383_amd import synth
from tests.exact import fr, limb_sum_diff


def _tiny_system(rng, n=3, terms=5, maxdeg=3):
    eqs = []
    for i in range(n):
        eq = [(synth.unit_complex(rng), {i: maxdeg}), (synth.unit_complex(rng), {})]
        for _ in range(terms - 2):
            k = int(rng.integers(1, n + 1))
            vs = rng.choice(n, size=k, replace=False)
            mono = {}
            budget = maxdeg
            for v in vs:
                if budget <= 0:
                    break
                e = int(rng.integers(1, budget + 1))
                mono[int(v)] = e
                budget -= e
            eq.append((synth.unit_complex(rng), mono))
        eqs.append(eq)
    return synth.system_from_terms(n, eqs)


def _sympy_system(s, xs):
    F = []
    for i in range(s.n_eq):
        expr = 0
        for c, mono in s.terms(i):
            cc = _q(Fraction(c.real)) + sp.I * _q(Fraction(c.imag))
            m = cc
            for v, e in mono:
                m = m * xs[v] ** e
            expr += m
        F.append(sp.expand(expr))
    return F


def _q(f: Fraction):
    return sp.Rational(f.numerator, f.denominator)


def _to_sym(limbs2L):
    return _q(fr(limbs2L[0])) + sp.I * _q(fr(limbs2L[1]))


def _cerr(got2L, exact):
    """Largest componentwise |got - exact| (exact rational difference, then float)."""
    er, ei = sp.re(exact), sp.im(exact)
    return max(abs(float(_q(fr(got2L[0])) - er)), abs(float(_q(fr(got2L[1])) - ei)))


@pytest.mark.parametrize("L", [1, 2, 4])
def test_eval_against_exact_sympy(L):
    rng = np.random.default_rng(10 + L)
    for trial in range(3):
        s = _tiny_system(rng, n=3, terms=6, maxdeg=3)
        xs = sp.symbols("x0:3")
        F = _sympy_system(s, xs)
        deg = s.degrees()
        gamma = synth.unit_complex(rng)
        t = float(rng.uniform(0, 1))
        x = synth.random_points(3, 2, L, rng)
        val, jac, sv, sj = oracle.eval_homotopy(s, L, x, np.full(2, t), gamma)
        G = _q(Fraction(gamma.real)) + sp.I * _q(Fraction(gamma.imag))
        T = _q(Fraction(t))
        H = [G * (1 - T) * (xs[i] ** int(deg[i]) - 1) + T * F[i] for i in range(3)]
        tol = 64 * 2.0 ** (-53 * L)
        for p in range(2):
            sub = {xs[j]: _to_sym(x[p, j]) for j in range(3)}
            for i in range(3):
                ex = sp.expand(H[i].subs(sub))
                assert _cerr(val[p, i], ex) <= tol * sv[p, i] + 1e-300
                for j in range(3):
                    exd = sp.expand(sp.diff(H[i], xs[j]).subs(sub))
                    assert _cerr(jac[p, i, j], exd) <= tol * sj[p, i, j] + 1e-300, (i, j)
                    if sj[p, i, j] == 0:
                        assert np.all(jac[p, i, j] == 0)


@pytest.mark.parametrize("L", [1, 2, 4])
def test_term_shapes_k0_k1_k2(L):
    # f = 2 + 3 x0 + x0^2 x1 (k = 0, 1, 2 terms), evaluated at exact points
    s = synth.system_from_terms(2, [[(2, {}), (3, {0: 1}), (1, {0: 2, 1: 1})],
                                    [(1j, {1: 1})]])
    x = np.zeros((1, 2, 2, L))
    x[0, 0, 0, 0], x[0, 0, 1, 0] = 0.5, -1.0   # x0 = 0.5 - i
    x[0, 1, 0, 0], x[0, 1, 1, 0] = 2.0, 0.25   # x1 = 2 + 0.25 i
    val, jac, _, _ = oracle.eval_homotopy(s, L, x, None)
    x0, x1 = 0.5 - 1j, 2 + 0.25j
    assert complex(val[0, 0, 0, 0], val[0, 0, 1, 0]) == 2 + 3 * x0 + x0 ** 2 * x1
    assert complex(jac[0, 0, 0, 0, 0], jac[0, 0, 0, 1, 0]) == 3 + 2 * x0 * x1
    assert complex(jac[0, 0, 1, 0, 0], jac[0, 0, 1, 1, 0]) == x0 ** 2
    assert complex(val[0, 1, 0, 0], val[0, 1, 1, 0]) == 1j * x1
    assert complex(jac[0, 1, 0, 0, 0], jac[0, 1, 0, 1, 0]) == 0
    assert complex(jac[0, 1, 1, 0, 0], jac[0, 1, 1, 1, 0]) == 1j


def test_finite_differences_real_direction():
    """Central differences along the real axis in quad double, exact difference
    of the limb sums: (F(x+h) - F(x-h)) / 2h = J + O(h^2), h = 2^-40."""
    rng = np.random.default_rng(20)
    s = synth.eval_dense(seed=123, n=5, terms_per_eq=8, k=3)
    L = 4
    x = synth.random_points(5, 1, L, rng, 0.7)
    t = np.array([0.3])
    gamma = synth.unit_complex(rng)
    val, jac, sv, sj = oracle.eval_homotopy(s, L, x, t, gamma)
    h = 2.0 ** -40
    for j in range(5):
        xp, xm = x.copy(), x.copy()
        xp[:, j, 0, 0] += h
        xm[:, j, 0, 0] -= h
        assert fr(xp[0, j, 0]) - fr(x[0, j, 0]) == Fraction(h)
        vp, _, _, _ = oracle.eval_homotopy(s, L, xp, t, gamma, jac=False, scales=False)
        vm, _, _, _ = oracle.eval_homotopy(s, L, xm, t, gamma, jac=False, scales=False)
        for i in range(5):
            for c in range(2):
                fd = (fr(vp[0, i, c]) - fr(vm[0, i, c])) / (2 * Fraction(h))
                assert float(abs(fd - fr(jac[0, i, j, c]))) <= 1e-20 * max(1.0, sj[0, i, j])


def test_finite_differences_tight_dd_differences():
    """Same check at much higher resolution: differences of QD values formed
    exactly, step 2^-40, truncation O(h^2) ~ 1e-24."""
    rng = np.random.default_rng(21)
    s = synth.eval_dense(seed=124, n=4, terms_per_eq=6, k=3)
    L = 4
    x = synth.random_points(4, 1, L, rng, 0.8)
    t = np.array([0.6])
    gamma = synth.unit_complex(rng)
    val, jac, sv, sj = oracle.eval_homotopy(s, L, x, t, gamma)
    h = 2.0 ** -40
    for j in range(4):
        xp, xm = x.copy(), x.copy()
        xp[:, j, 1, 0] += h   # step along the imaginary axis: dF = i * dF/dx * h
        xm[:, j, 1, 0] -= h
        vp, _, _, _ = oracle.eval_homotopy(s, L, xp, t, gamma, jac=False, scales=False)
        vm, _, _, _ = oracle.eval_homotopy(s, L, xm, t, gamma, jac=False, scales=False)
        for i in range(4):
            dre = fr(vp[0, i, 0]) - fr(vm[0, i, 0])
            dim = fr(vp[0, i, 1]) - fr(vm[0, i, 1])
            # (F(x+ih) - F(x-ih)) / (2h) = i J  =>  J = (dim - i dre) / (2h)
            jr = dim / (2 * Fraction(h))
            ji = -dre / (2 * Fraction(h))
            err = max(abs(jr - fr(jac[0, i, j, 0])), abs(ji - fr(jac[0, i, j, 1])))
            assert float(err) <= 1e-20 * max(1.0, sj[0, i, j])


@pytest.mark.parametrize("L", [1, 2])
def test_euler_identity_homogeneous(L):
    """All terms of equation i have the same degree d_i: sum_j x_j J_ij = d_i f_i."""
    rng = np.random.default_rng(30)
    n = 5
    eqs = []
    for i in range(n):
        d = 2 + i % 3
        eq = []
        for _ in range(7):
            mono = {}
            for _ in range(d):
                v = int(rng.integers(0, n))
                mono[v] = mono.get(v, 0) + 1
            eq.append((synth.unit_complex(rng), mono))
        eqs.append(eq)
    s = synth.system_from_terms(n, eqs)
    x = synth.random_points(n, 3, L, rng)
    val, jac, sv, sj = oracle.eval_homotopy(s, L, x, None)
    V = val[..., 0, 0] + 1j * val[..., 1, 0]
    J = jac[..., 0, 0] + 1j * jac[..., 1, 0]
    X = x[..., 0, 0] + 1j * x[..., 1, 0]
    lhs = np.einsum("pij,pj->pi", J, X)
    d = np.array([2 + i % 3 for i in range(n)])
    rhs = d[None, :] * V
    assert np.max(np.abs(lhs - rhs) / (1 + np.abs(rhs))) < 1e-12


@pytest.mark.parametrize("L", [1, 2, 4])
def test_t0_t1_and_start_zeros(L):
    rng = np.random.default_rng(40)
    s = synth.tracking_cubic()
    gamma = synth.gamma_of(s)
    x = synth.random_points(s.n_var, 3, L, rng)
    v1, j1, _, _ = oracle.eval_homotopy(s, L, x, np.ones(3), gamma)
    vf, jf, _, _ = oracle.eval_homotopy(s, L, x, None, gamma)
    # t = 1: f alone (scaling by 1 and gamma * 0 are exact): same values
    assert np.all(limb_sum_diff(v1, vf) == 0) and np.all(limb_sum_diff(j1, jf) == 0)
    # t = 0: gamma * (x_i^3 - 1), Jacobian diagonal gamma * 3 x_i^2
    v0, j0, sv, _ = oracle.eval_homotopy(s, L, x, np.zeros(3), gamma)
    X = x[..., 0, 0] + 1j * x[..., 1, 0]
    V0 = v0[..., 0, 0] + 1j * v0[..., 1, 0]
    assert np.allclose(V0, gamma * (X ** 3 - 1), rtol=1e-13, atol=1e-13)
    J0 = j0[..., 0, 0] + 1j * j0[..., 1, 0]
    for p in range(3):
        assert np.allclose(J0[p], np.diag(gamma * 3 * X[p] ** 2), rtol=1e-13, atol=1e-15)
    # roots of unity are zeros of g: H(x0, 0) ~ 0 at every start solution
    deg = oracle.degrees(s)
    for pidx in (0, 1, 100, 6560):
        xs = oracle.start_solution(L, deg, pidx)[None]
        v, _, sv, _ = oracle.eval_homotopy(s, L, xs, np.zeros(1), gamma, jac=False)
        for i in range(s.n_eq):
            assert abs(float(fr(v[0, i, 0]))) <= 8 * 2.0 ** (-52 * L) * sv[0, i]
            assert abs(float(fr(v[0, i, 1]))) <= 8 * 2.0 ** (-52 * L) * sv[0, i]


def test_general_start_system_matches_total_degree():
    """A start system passed explicitly as x_i^{d_i} - 1 equals the built-in one."""
    s = synth.tracking_small()
    deg = s.degrees()
    g = synth.system_from_terms(s.n_var, [[(1, {i: int(deg[i])}), (-1, {})] for i in range(s.n_eq)])
    rng = np.random.default_rng(41)
    x = synth.random_points(s.n_var, 4, 2, rng)
    t = rng.uniform(0, 1, 4)
    gamma = synth.gamma_of(s)
    a = oracle.eval_homotopy(s, 2, x, t, gamma)
    b = oracle.eval_homotopy(s, 2, x, t, gamma, start=g)
    for u, w in zip(a[:2], b[:2]):
        d = np.abs((u.sum(-1) - w.sum(-1)))
        assert np.max(d) < 1e-28 * (1 + np.max(np.abs(u)))
