"""Pins of the oracle's start solutions and path tracker.

Only endpoints are pinned (the step sequence is a heuristic and parity-unpinned):
* closed-form roots of unity and the mixed-radix path numbering;
* f = g: every path stays at its start point;
* decoupled f_i = x_i^{d_i} - c_i: closed-form path x_i(t)^{d_i} =
  (gamma(1-t) + t c_i) / (gamma(1-t) + t), endpoint the d_i-th root of c_i on the
  branch continued from the start point (argument unwrapped on a fine t grid);
* n = 1: the set of endpoints equals numpy.roots;
* Bezout count: B paths succeed with B distinct endpoints;
* residual of polished endpoints is at the rounding level;
* forced failures: a path to infinity, NaN start, h_min > h_init, max_steps,
  singular Jacobian.
"""
from fractions import Fraction

import os

import numpy as np
import pytest

import oracle
from paper_1505_00383_amd import synth
from tests.exact import frc, limb_sum_diff
from tests.starts import diagonal_roots, diagonal_start

U = {1: 2.0 ** -53, 2: 2.0 ** -104, 4: 2.0 ** -208}


def _cx(x):
    """[..., 2, L] -> complex (hi limbs)."""
    return x[..., 0, 0] + 1j * x[..., 1, 0]


@pytest.mark.parametrize("L", [1, 2, 4])
def test_start_solutions_closed_form(L):
    deg = np.array([2, 3, 2, 3], dtype=np.int32)
    B = int(np.prod(deg))
    seen = set()
    for p in range(B):
        x = oracle.start_solution(L, deg, p)
        # little-endian mixed radix
        k, q = [], p
        for d in deg:
            k.append(q % d)
            q //= d
        ref = np.exp(2j * np.pi * np.array(k) / deg)
        assert np.max(np.abs(_cx(x) - ref)) <= 1e-15
        for i, d in enumerate(deg):
            re, im = frc(x[i])
            z = (re, im)
            # z^d exactly in rationals
            pr, pi_ = Fraction(1), Fraction(0)
            for _ in range(int(d)):
                pr, pi_ = pr * z[0] - pi_ * z[1], pr * z[1] + pi_ * z[0]
            assert abs(pr - 1) <= 8 * Fraction(U[L]) and abs(pi_) <= 8 * Fraction(U[L])
            if d == 2:
                assert pi_ == 0 and pr == 1   # +-1 exactly
        seen.add(tuple(np.round(_cx(x), 12)))
    assert len(seen) == B


@pytest.mark.parametrize("L", [1, 2])
def test_f_equals_g_paths_stay_put(L):
    n = 3
    deg = [2, 3, 2]
    s = synth.system_from_terms(n, [[(1, {i: deg[i]}), (-1, {})] for i in range(n)])
    gamma = complex(np.cos(1.1), np.sin(1.1))
    r = oracle.track(s, gamma, range(12), oracle.Opts(prec=L))
    assert np.all(r["status"] == 1)
    for p in range(12):
        x0 = oracle.start_solution(L, np.array(deg, dtype=np.int32), p)
        assert np.max(np.abs(_cx(r["x"][p]) - _cx(x0))) <= 1e-14


def _golden(name):
    out = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as f:
        for ln in f:
            if ln.strip() and not ln.startswith("#"):
                k, v = ln.split()
                out[k] = int(v)
    return out


@pytest.mark.parametrize("L", [1, 2, 4])
def test_f_equals_g_step_sequence_by_hand(L):
    """On f = g every step is accepted with one Newton step, so the step count
    is what the step-size rule gives by hand (tests/golden/
    step_sequence_f_equals_g.txt): a wrong expansion count, factor or cap, or
    a rejected step, changes it."""
    want = _golden("step_sequence_f_equals_g.txt")
    n = 3
    deg = [2, 3, 2]
    s = synth.system_from_terms(n, [[(1, {i: deg[i]}), (-1, {})] for i in range(n)])
    gamma = complex(np.cos(1.1), np.sin(1.1))
    r = oracle.track(s, gamma, range(4), oracle.Opts(prec=L))
    assert np.all(r["status"] == 1)
    assert np.all(r["steps"] == want["steps"])
    assert np.all(r["newton"] == want["newton"])


def _branch_endpoint(gamma, c, d, x0, steps=20000):
    t = np.linspace(0.0, 1.0, steps + 1)
    w = (gamma * (1 - t) + t * c) / (gamma * (1 - t) + t)
    ang = np.unwrap(np.angle(w))
    ang += (np.angle(x0 ** d) - ang[0])            # w(0) = 1 = x0^d
    theta0 = np.angle(x0)
    # x(t) = |w|^(1/d) exp(i (theta0 + (ang - ang0)/d))
    return np.abs(w[-1]) ** (1.0 / d) * np.exp(1j * (theta0 + (ang[-1] - ang[0]) / d))


@pytest.mark.parametrize("order", [1, 4])
@pytest.mark.parametrize("L", [1, 2])
def test_decoupled_closed_form(L, order):
    rng = np.random.default_rng(7)
    n = 3
    deg = np.array([3, 2, 3], dtype=np.int32)
    cs = [0.5 * synth.unit_complex(rng) * (1 + rng.uniform()) for _ in range(n)]
    s = synth.system_from_terms(n, [[(1, {i: int(deg[i])}), (-cs[i], {})] for i in range(n)])
    gamma = synth.unit_complex(rng)
    B = int(np.prod(deg))
    r = oracle.track(s, gamma, range(B), oracle.Opts(prec=L, predictor_order=order))
    assert np.all(r["status"] == 1)
    for p in range(B):
        x0 = _cx(oracle.start_solution(1, deg, p))
        for i in range(n):
            ref = _branch_endpoint(gamma, cs[i], int(deg[i]), x0[i])
            assert abs(_cx(r["x"][p])[i] - ref) <= 1e-9, (p, i)


def test_univariate_against_numpy_roots():
    rng = np.random.default_rng(11)
    d = 6
    coeffs = [synth.unit_complex(rng) for _ in range(d + 1)]  # x^d ... x^0
    s = synth.system_from_terms(1, [[(coeffs[d - e], {0: e} if e else {}) for e in range(d + 1)]])
    gamma = synth.unit_complex(rng)
    r = oracle.track(s, gamma, range(d), oracle.Opts(prec=2))
    assert np.all(r["status"] == 1)
    got = np.sort_complex(_cx(r["x"][:, 0]))
    ref = np.roots(coeffs)
    for z in got:
        assert np.min(np.abs(ref - z)) <= 1e-12
    for z in ref:
        assert np.min(np.abs(got - z)) <= 1e-12


def _residual_ok(s, r, L, c=256.0):
    X = r["x"]
    val, _, sv, _ = oracle.eval_homotopy(s, L, X, None, jac=False)
    res = np.abs(val.sum(-1)).max(-1)   # [p, i]
    return np.all(res <= c * U[L] * np.maximum(sv, 1.0))


@pytest.mark.parametrize("order", [1, 4])
@pytest.mark.parametrize("L", [1, 2])
def test_bezout_count_small(L, order):
    s = synth.tracking_small()
    r = oracle.track(s, synth.gamma_of(s), range(8), oracle.Opts(prec=L, predictor_order=order))
    assert np.all(r["status"] == 1)
    E = _cx(r["x"])
    for a in range(8):
        for b in range(a + 1, 8):
            assert np.max(np.abs(E[a] - E[b])) > 1e-6
    assert _residual_ok(s, r, L)


@pytest.mark.parametrize("order", [1, 4])
def test_bezout_count_cubic_n3(order):
    """n = 3, degree 3 per equation (x_i^3, 1, 6 random others): 27 distinct endpoints."""
    rng = np.random.default_rng(12)
    eqs = [synth._equation_with_anchor(rng, [0, 1, 2], i, 3, 8) for i in range(3)]
    s = synth.system_from_terms(3, eqs)
    r = oracle.track(s, synth.unit_complex(rng), range(27), oracle.Opts(prec=1, predictor_order=order))
    assert np.all(r["status"] == 1)
    E = _cx(r["x"])
    d = np.abs(E[:, None, :] - E[None, :, :]).max(-1) + np.eye(27)
    assert d.min() > 1e-6
    assert _residual_ok(s, r, 1)


def test_mixed_and_plain_agree_double_double():
    s = synth.tracking_small()
    g = synth.gamma_of(s)
    plain = oracle.track(s, g, range(8), oracle.Opts(prec=2, mixed=0))
    mixed = oracle.track(s, g, range(8), oracle.Opts(prec=2, mixed=1))
    assert np.all(plain["status"] == 1) and np.all(mixed["status"] == 1)
    from tests.exact import limb_sum_diff
    d = np.abs(limb_sum_diff(plain["x"], mixed["x"])).max()
    assert d <= 1e-24 * max(1.0, np.abs(_cx(plain["x"])).max())
    assert _residual_ok(s, mixed, 2)


def test_forced_divergence_exactly_one():
    # f = 0 x^2 + x - 1 keeps degree 2 (start x^2 - 1) but has one finite root
    s = synth.system_from_terms(1, [[(0.0, {0: 2}), (1.0, {0: 1}), (-1.0, {})]])
    gamma = complex(np.cos(0.7), np.sin(0.7))
    r = oracle.track(s, gamma, range(2), oracle.Opts(prec=1))
    reasons = sorted(oracle.REASONS[int(v)] for v in r["reason"])
    assert reasons == ["DIVERGED", "SUCCESS"]
    ok = int(np.argmax(r["status"] == 1))
    assert abs(_cx(r["x"][ok, 0]) - 1.0) <= 1e-12


def test_forced_failures():
    s = synth.tracking_small()
    g = synth.gamma_of(s)
    deg = oracle.degrees(s)
    x0 = oracle.start_solution(1, deg, 0)
    xn = x0.copy()
    xn[1, 0, 0] = np.nan
    assert oracle.REASONS[oracle.track_path(s, g, xn, oracle.Opts())["reason"]] == "NAN"
    r = oracle.track_path(s, g, x0, oracle.Opts(h_min=0.1, h_init=0.01))
    assert oracle.REASONS[r["reason"]] == "STEP_UNDERFLOW" and r["status"] == -1
    r = oracle.track_path(s, g, x0, oracle.Opts(max_steps=1))
    assert oracle.REASONS[r["reason"]] == "MAX_STEPS" and r["status"] == -1
    # at x = 0 both g and f = x_i^2 - 1 have a zero Jacobian: every solve is singular
    f = synth.system_from_terms(2, [[(1, {0: 2}), (-1, {})], [(1, {1: 2}), (-1, {})]])
    r = oracle.track_path(f, g, np.zeros((2, 2, 1)), oracle.Opts())
    assert oracle.REASONS[r["reason"]] == "SINGULAR" and r["status"] == -1


@pytest.mark.parametrize("L", [1, 2, 4])
@pytest.mark.parametrize("m", [2, 3, 4])
def test_extrapolation_exact_on_polynomials(L, m):
    """The predictor of order m reproduces every polynomial path of degree m
    (up to the FP64 weights) and misses one of degree m + 1: checks the
    nodes, the weights and the sum, including the node count."""
    rng = np.random.default_rng(100 + 10 * m + L)
    n = 3
    # dyadic nodes (previous points at decreasing t) and coefficients, so
    # every sample value is exact in double
    T = np.array([0.5 - 0.0625 * j for j in range(m + 1)])
    t1 = 0.5 + 0.125
    for deg, exact in ((m, True), (m + 1, False)):
        cre = rng.integers(-8, 9, size=(n, deg + 1)) / 8.0
        cim = rng.integers(-8, 9, size=(n, deg + 1)) / 8.0
        cre[:, deg] += np.where(cre[:, deg] == 0, 1.0, 0.0)   # keep the top degree
        P = lambda tt: (np.polyval(cre[:, ::-1].T, tt) + 1j * np.polyval(cim[:, ::-1].T, tt))
        X = np.zeros((m + 1, n, 2, L))
        for j in range(m + 1):
            z = P(T[j])
            X[j, :, 0, 0], X[j, :, 1, 0] = z.real, z.imag
        got = oracle.extrapolate(L, T, X, t1)
        ref = P(t1)
        err = np.abs((got[:, 0, :].sum(-1) + 1j * got[:, 1, :].sum(-1)) - ref).max()
        scale = max(1.0, np.abs(ref).max())
        if exact:
            assert err <= 1e-13 * scale, (deg, err)
        else:
            assert err > 1e-6, (deg, err)


def test_extrapolation_order_one_is_the_secant():
    """With two nodes the Lagrange form is the secant x + r (x - xp)."""
    L = 2
    T = np.array([0.4, 0.3])
    X = np.zeros((2, 1, 2, L))
    X[0, 0, 0, 0], X[0, 0, 1, 0] = 1.25, -0.5
    X[1, 0, 0, 0], X[1, 0, 1, 0] = 0.75, 0.25
    got = oracle.extrapolate(L, T, X, 0.55)
    r = (0.55 - 0.4) / (0.4 - 0.3)
    ref = complex(1.25, -0.5) + r * (complex(1.25, -0.5) - complex(0.75, 0.25))
    assert abs(complex(got[0, 0].sum(), got[0, 1].sum()) - ref) <= 1e-15


# ---------------------------------------------------------------------------
# Quad double (L = 4): the tracker's own pins at QD accuracy
# ---------------------------------------------------------------------------
def _mpc_of(limbs_cx):
    """exact value of a [2][L] limb complex as an mpmath number (working
    precision set by the caller)."""
    import mpmath
    re, im = frc(limbs_cx)
    return mpmath.mpc(mpmath.mpf(re.numerator) / re.denominator,
                      mpmath.mpf(im.numerator) / im.denominator)


@pytest.mark.parametrize("mixed", [0, 1])
def test_decoupled_closed_form_quad_double(mixed):
    """f_i = x_i^{d_i} - c_i at L = 4: every endpoint is the d_i-th root of c_i
    on the branch continued from its start point (Section 2's paths), to
    1e-50 relative.  The branch is chosen by the FP64 unwrapped continuation;
    the root itself is computed by mpmath at 80 digits from the exact FP64
    value of c_i, so the reference owes nothing to the oracle's arithmetic."""
    import mpmath
    mpmath.mp.dps = 80
    rng = np.random.default_rng(23)
    n = 3
    deg = np.array([3, 2, 3], dtype=np.int32)
    cs = [0.5 * synth.unit_complex(rng) * (1 + rng.uniform()) for _ in range(n)]
    s = synth.system_from_terms(n, [[(1, {i: int(deg[i])}), (-cs[i], {})] for i in range(n)])
    gamma = synth.unit_complex(rng)
    B = int(np.prod(deg))
    r = oracle.track(s, gamma, range(B), oracle.Opts(prec=4, mixed=mixed))
    assert np.all(r["status"] == 1)
    worst = 0.0
    for p in range(B):
        x0 = _cx(oracle.start_solution(1, deg, p))
        for i in range(n):
            approx = _branch_endpoint(gamma, cs[i], int(deg[i]), x0[i])
            c = mpmath.mpc(cs[i].real, cs[i].imag)
            d = int(deg[i])
            roots = [mpmath.root(c, d, m) for m in range(d)]   # all d-th roots
            ref = min(roots, key=lambda z: abs(complex(z) - approx))
            got = _mpc_of(r["x"][p, i])
            err = float(abs(got - ref) / max(1, abs(ref)))
            worst = max(worst, err)
            assert err <= 1e-50, (p, i, err)
    print(f"decoupled QD mixed={mixed}: worst relative endpoint error {worst:.1e}")


def test_f_equals_g_paths_stay_put_quad_double():
    n = 3
    deg = [2, 3, 2]
    s = synth.system_from_terms(n, [[(1, {i: deg[i]}), (-1, {})] for i in range(n)])
    gamma = complex(np.cos(1.1), np.sin(1.1))
    r = oracle.track(s, gamma, range(12), oracle.Opts(prec=4))
    assert np.all(r["status"] == 1)
    for p in range(12):
        x0 = oracle.start_solution(4, np.array(deg, dtype=np.int32), p)
        d = np.abs(limb_sum_diff(r["x"][p], x0)).max()
        assert d <= 1e-60, (p, d)


def test_quad_double_residual_and_mixed_agreement():
    """The n = 3, degree-2 workload at L = 4: 8 distinct endpoints, residual
    |f(x*)| <= 256 u_QD S at every polished endpoint (polish target 8 u_QD),
    and the mixed scheme (FP64 Newton solves) ends within 1e-48 of the plain
    quad-double track."""
    s = synth.tracking_small()
    g = synth.gamma_of(s)
    plain = oracle.track(s, g, range(8), oracle.Opts(prec=4, mixed=0))
    mixed = oracle.track(s, g, range(8), oracle.Opts(prec=4, mixed=1))
    assert np.all(plain["status"] == 1) and np.all(mixed["status"] == 1)
    assert _residual_ok(s, plain, 4) and _residual_ok(s, mixed, 4)
    E = _cx(plain["x"])
    for a in range(8):
        for b in range(a + 1, 8):
            assert np.max(np.abs(E[a] - E[b])) > 1e-6
    d = np.abs(limb_sum_diff(plain["x"], mixed["x"])).max()
    assert d <= 1e-48 * max(1.0, np.abs(E).max()), d


def test_singular_flag_quad_double():
    """At x = 0 the Jacobian of x_i^2 - 1 and of the start system vanish: the
    quad-double MGS (threshold 2^-200 ||A||_F) flags every solve singular."""
    f = synth.system_from_terms(2, [[(1, {0: 2}), (-1, {})], [(1, {1: 2}), (-1, {})]])
    g = synth.gamma_of(synth.tracking_small())
    r = oracle.track_path(f, g, np.zeros((2, 2, 4)), oracle.Opts(prec=4))
    assert oracle.REASONS[r["reason"]] == "SINGULAR" and r["status"] == -1


# ---------------------------------------------------------------------------
# Explicit start systems g (Eq. (1) allows any g with known roots)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("L", [1, 2, 4])
def test_custom_start_f_equals_g_stays_put(L):
    """f = g for a start system that is not x^d - 1: H = (gamma(1-t) + t) g, so
    every path stays at its start point, which is a root of g only up to the
    rounding of its limbs; the endpoint must be that root to ~u_L."""
    rng = np.random.default_rng(31)
    deg = [2, 3, 2]
    g, a, b = diagonal_start(rng, deg)
    paths = np.arange(12)
    X0 = diagonal_roots(a, b, deg, L, paths)
    r = oracle.track(g, complex(np.cos(0.4), np.sin(0.4)), paths, oracle.Opts(prec=L), start=g, x0=X0)
    assert np.all(r["status"] == 1)
    d = np.abs(limb_sum_diff(r["x"], X0)).max()
    assert d <= 64 * U[L], d


@pytest.mark.parametrize("L", [1, 2])
def test_custom_start_reaches_the_same_endpoints(L):
    """The endpoints of the n = 3, degree-2 workload do not depend on the start
    system: tracked from a diagonal start system with random coefficients they
    are, as a set, the endpoints tracked from x_i^2 - 1 (and each has a
    residual at the rounding level)."""
    s = synth.tracking_small()
    gam = synth.gamma_of(s)
    rng = np.random.default_rng(41)
    deg = [2, 2, 2]
    g, a, b = diagonal_start(rng, deg)
    X0 = diagonal_roots(a, b, deg, L, np.arange(8))
    custom = oracle.track(s, gam, np.arange(8), oracle.Opts(prec=L), start=g, x0=X0)
    total = oracle.track(s, gam, range(8), oracle.Opts(prec=L))
    assert np.all(custom["status"] == 1) and np.all(total["status"] == 1)
    assert _residual_ok(s, custom, L)
    Ec, Et = _cx(custom["x"]), _cx(total["x"])
    for z in Ec:
        assert np.min(np.abs(Et - z).max(-1)) <= 1e-10
    for z in Et:
        assert np.min(np.abs(Ec - z).max(-1)) <= 1e-10


# ---------------------------------------------------------------------------
# The residual half of the corrector's convergence test, and the endpoint check
# ---------------------------------------------------------------------------
def test_residual_test_binds():
    """Section 2 ends the corrector when the residual AND the update are small.
    With tol_res so small that no residual can meet it, no step converges and
    every path ends by step-size underflow; with the default the same paths
    all succeed; with tol_res = inf the update test alone decides and, on this
    well-conditioned workload, gives the same endpoints."""
    s = synth.tracking_small()
    g = synth.gamma_of(s)
    r = oracle.track(s, g, range(4), oracle.Opts(prec=1, tol_res=1e-300))
    assert all(oracle.REASONS[int(v)] == "STEP_UNDERFLOW" for v in r["reason"])
    a = oracle.track(s, g, range(8), oracle.Opts(prec=2))
    b = oracle.track(s, g, range(8), oracle.Opts(prec=2, tol_res=float("inf")))
    assert np.all(a["status"] == 1) and np.all(b["status"] == 1)
    assert np.abs(limb_sum_diff(a["x"], b["x"])).max() <= 1e-28


def test_polished_endpoint_beyond_diverge_norm_fails():
    """A polished endpoint must lie within diverge_norm.  f = -(x - 2)(x - 4)
    is concave on the real axis, so Newton from the start point x = 1 climbs
    to the root 2 from below: with one step straight to t = 1 and a loose
    corrector (tol_dx = 0.5, one Newton step) the point accepted at t = 1 is
    x = 1.75, inside diverge_norm = 1.9; the polish then reaches x = 2, which
    must end the path as DIVERGED rather than report success."""
    f = synth.system_from_terms(1, [[(-1, {0: 2}), (6, {0: 1}), (-8, {})]])
    gamma = complex(np.cos(0.3), np.sin(0.3))
    loose = dict(prec=1, tol_dx=0.5, tol_res=float("inf"), h_init=1.0, h_max=1.0, max_newton=1)
    x0 = oracle.start_solution(1, np.array([2], dtype=np.int32), 0)      # x = 1
    assert _cx(x0)[0] == 1.0
    r1 = oracle.track_path(f, gamma, x0, oracle.Opts(**loose))
    assert r1["status"] == 1 and r1["steps"] == 1 and abs(_cx(r1["x"])[0] - 2.0) <= 1e-14
    r2 = oracle.track_path(f, gamma, x0, oracle.Opts(**loose, diverge_norm=1.9))
    assert r2["status"] == -1 and oracle.REASONS[r2["reason"]] == "DIVERGED"
