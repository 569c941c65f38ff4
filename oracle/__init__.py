"""CPU oracle for the many-path homotopy hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product (the HIP library and its
Python binding) never imports it, and the two share no code.

The arithmetic lives in ``oracle.c`` (exact floating-point expansions cut to L
limbs; Dekker/Veltkamp products, no FMA).  This module only marshals numpy
arrays through ctypes and loops over points/paths.

Parity status of every exported function (what pins it, in ``tests/``):

* ``mp_op`` / ``cx_op``          -- pinned: exact ``fractions.Fraction`` results.
* ``eval_homotopy``              -- pinned: exact Fraction evaluation of tiny
  systems, central finite differences, Euler's identity, t = 0 / t = 1 special
  cases, the roots-of-unity zeros of the start system.
* ``mgs``                        -- pinned: ``numpy.linalg.lstsq``, mpmath QR at
  high precision, orthonormality of Q, the singular flag.
* ``start_solution``             -- pinned: closed form, x_i^{d_i} = 1 in Fraction.
* ``track_path`` / ``track``     -- pinned: f = g invariance (total-degree and
  explicit start systems, L = 1, 2, 4), decoupled closed form (to 1e-9 in D/DD,
  to 1e-50 against 80-digit mpmath roots in QD, plain and mixed), n = 1 against
  ``numpy.roots``, Bezout count with distinct endpoints, endpoint residuals
  (<= 256 u_L S, L = 1, 2, 4), mixed vs plain agreement (1e-24 DD, 1e-48 QD),
  endpoints independent of the start system, the residual half of the
  convergence test, the endpoint check after the polish, forced failures.
  The step sequence itself is pinned only on f = g (a hand-derived step count);
  on moving paths it is parity unpinned (only endpoints are pinned).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, asdict

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_LIB_DIR, "liboracle.so")

REASONS = {0: "NONE", 1: "SUCCESS", 2: "DIVERGED", 3: "STEP_UNDERFLOW", 4: "MAX_STEPS",
           5: "SINGULAR", 6: "NAN"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 -ffp-contract=off (no fast-math)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    os.makedirs(_LIB_DIR, exist_ok=True)
    tmp = _LIB + f".tmp{os.getpid()}"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
                           "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int, ctypes.c_int64
        L.ora_mp_op.argtypes = [i32, i32, P, P, P]
        L.ora_cx_op.argtypes = [i32, i32, P, P, P]
        L.ora_degrees.argtypes = [i32, i32, P, P, P, P, P, P]
        L.ora_eval.argtypes = [i32, i32, i32, P, P, P, P, P, i32, P, P, P, P, P, P, i32, P, i64,
                               P, P, P, P, P]
        L.ora_mgs.argtypes = [i32, i32, i32, P, P, P, P]
        L.ora_mgs.restype = i32
        L.ora_start_solution.argtypes = [i32, i32, P, i64, P]
        L.ora_start_solution.restype = i32
        L.ora_track_path.argtypes = [i32, P, i32, i32, P, P, P, P, P, i32, P, P, P, P, P, P, P, P,
                                     P, P, P, P]
        L.ora_extrapolate.argtypes = [i32, i32, i32, P, P, ctypes.c_double, P]
        L.ora_track_path.restype = i32
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# ---------------------------------------------------------------------------
# arithmetic probes
# ---------------------------------------------------------------------------
MP_ADD, MP_SUB, MP_MUL, MP_DIV, MP_SQRT = range(5)
CX_ADD, CX_MUL, CX_CMUL = range(3)


def mp_op(L: int, op: int, a, b=None) -> np.ndarray:
    a = _c(a, np.float64)
    b = None if b is None else _c(b, np.float64)
    out = np.zeros(L)
    lib().ora_mp_op(L, op, _p(a), _p(b), _p(out))
    return out


def cx_op(L: int, op: int, a, b) -> np.ndarray:
    a = _c(a, np.float64)
    b = _c(b, np.float64)
    out = np.zeros((2, L))
    lib().ora_cx_op(L, op, _p(a), _p(b), _p(out))
    return out


# ---------------------------------------------------------------------------
# evaluation
# ---------------------------------------------------------------------------
def _sys_args(s):
    return (_c(s.eq_term_off, np.int32), _c(s.term_fac_off, np.int32), _c(s.fac_var, np.int32),
            _c(s.fac_exp, np.int32), _c(s.coef, np.float64))


def degrees(s) -> np.ndarray:
    arrs = _sys_args(s)
    d = np.zeros(s.n_eq, dtype=np.int32)
    lib().ora_degrees(s.n_eq, s.n_var, *[_p(a) for a in arrs], _p(d))
    return d


def eval_homotopy(s, L: int, x, t=None, gamma=1.0 + 0j, start=None, jac: bool = True,
                  scales: bool = True):
    """H(x,t) = gamma (1-t) g(x) + t f(x) and dH/dx at every point (Eq. (1)).

    x: [npts, n_var, 2, L]; t: [npts] or None (t = 1: f alone).
    Returns (val [npts,n_eq,2,L], jac [npts,n_eq,n_var,2,L] or None,
             sv [npts,n_eq], sj [npts,n_eq,n_var]) -- sv/sj are FP64 magnitude
    bounds sum |c(t)| |x^a| used to scale parity tolerances."""
    x = _c(x, np.float64)
    npts = x.shape[0]
    assert x.shape[1:] == (s.n_var, 2, L)
    arrs = _sys_args(s)
    if start is not None:
        garrs = _sys_args(start)
    else:
        garrs = (None,) * 5
    tt = None if t is None else _c(np.broadcast_to(np.asarray(t, dtype=np.float64), (npts,)), np.float64)
    g = np.array([complex(gamma).real, complex(gamma).imag])
    val = np.zeros((npts, s.n_eq, 2, L))
    jm = np.zeros((npts, s.n_eq, s.n_var, 2, L)) if jac else None
    sv = np.zeros((npts, s.n_eq)) if scales else None
    sj = np.zeros((npts, s.n_eq, s.n_var)) if (scales and jac) else None
    lib().ora_eval(L, s.n_eq, s.n_var, *[_p(a) for a in arrs], 1 if start is not None else 0,
                   *[_p(a) for a in garrs], _p(g), 0 if tt is None else 1, _p(tt), npts, _p(x),
                   _p(val), _p(jm), _p(sv), _p(sj))
    return val, jm, sv, sj


def eval_threaded(s, L, x, t=None, gamma=1.0 + 0j, threads: int = 1, jac=True, scales=False):
    """Same as eval_homotopy, split over contiguous point ranges on host threads
    (ctypes releases the GIL during the call)."""
    npts = x.shape[0]
    if threads <= 1 or npts < 2:
        return eval_homotopy(s, L, x, t, gamma, jac=jac, scales=scales)
    bounds = np.linspace(0, npts, threads + 1).astype(int)
    tt = None if t is None else np.broadcast_to(np.asarray(t, dtype=np.float64), (npts,))

    def work(k):
        a, b = bounds[k], bounds[k + 1]
        return eval_homotopy(s, L, x[a:b], None if tt is None else tt[a:b], gamma, jac=jac,
                             scales=scales)

    with ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(work, range(threads)))
    val = np.concatenate([p[0] for p in parts])
    jm = np.concatenate([p[1] for p in parts]) if jac else None
    return val, jm, None, None


# ---------------------------------------------------------------------------
# least squares
# ---------------------------------------------------------------------------
def mgs(L: int, A, b, want_q: bool = False):
    """Least squares A dx = b by MGS on [A | b] in L limbs.
    A: [m, n, 2, L], b: [m, 2, L].  Returns (dx [n,2,L] or None, singular, Q)."""
    A = _c(A, np.float64)
    b = _c(b, np.float64)
    m, n = A.shape[0], A.shape[1]
    dx = np.zeros((n, 2, L))
    q = np.zeros((m, n, 2, L)) if want_q else None
    sing = lib().ora_mgs(L, m, n, _p(A), _p(b), _p(dx), _p(q))
    return (None if sing else dx), bool(sing), q


# ---------------------------------------------------------------------------
# start solutions and tracking
# ---------------------------------------------------------------------------
def start_solution(L: int, deg, p: int) -> np.ndarray:
    deg = _c(deg, np.int32)
    x = np.zeros((len(deg), 2, L))
    if lib().ora_start_solution(L, len(deg), _p(deg), int(p), _p(x)):
        raise ValueError("no closed-form root of unity for these degrees")
    return x


@dataclass
class Opts:
    prec: int = 1
    mixed: int = 0
    predictor_order: int = 1
    max_newton: int = 3
    expand_after: int = 3
    polish_max: int = 8
    h_init: float = 0.01
    h_min: float = 1e-10
    h_max: float = 0.1
    shrink: float = 0.5
    expand: float = 1.5
    tol_dx: float = 1e-8
    diverge_norm: float = 1e8
    polish_tol: float = -1.0  # < 0 selects 8 u_L
    max_steps: int = 100_000
    tol_res: float = 1e-6     # residual test ||H|| <= tol_res ||J||_F max(1, ||x||)


class _COpts(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("mixed", ctypes.c_int32),
                ("predictor_order", ctypes.c_int32), ("max_newton", ctypes.c_int32),
                ("expand_after", ctypes.c_int32), ("polish_max", ctypes.c_int32),
                ("h_init", ctypes.c_double), ("h_min", ctypes.c_double),
                ("h_max", ctypes.c_double), ("shrink", ctypes.c_double),
                ("expand", ctypes.c_double), ("tol_dx", ctypes.c_double),
                ("diverge_norm", ctypes.c_double), ("polish_tol", ctypes.c_double),
                ("max_steps", ctypes.c_int64), ("tol_res", ctypes.c_double)]


def unit_roundoff(L: int) -> float:
    return {1: 2.0 ** -53, 2: 2.0 ** -104, 4: 2.0 ** -208}[L]


def _copts(o: Opts) -> _COpts:
    d = asdict(o)
    if d["polish_tol"] < 0:
        d["polish_tol"] = 8.0 * unit_roundoff(o.prec)
    return _COpts(**d)


def extrapolate(L: int, T, X, t1: float):
    """Predictor of order m = len(T) - 1 (Section 2): the interpolant of the
    points (T[j], X[j]) evaluated at t1.  X: [m+1, n, 2, L]."""
    T = _c(T, np.float64)
    X = _c(X, np.float64)
    m, n = len(T) - 1, X.shape[1]
    out = np.zeros((n, 2, L))
    lib().ora_extrapolate(L, m, n, _p(T), _p(X), float(t1), _p(out))
    return out


def track_path(s, gamma, x0, opts: Opts, start=None):
    """Track one path of gamma(1-t)g + t f from the start point x0 [n,2,L];
    g is ``start`` or, when None, the total-degree start system x_i^{d_i} - 1."""
    L = opts.prec
    x = _c(x0, np.float64).copy()
    assert x.shape == (s.n_var, 2, L)
    arrs = _sys_args(s)
    garrs = _sys_args(start) if start is not None else (None,) * 5
    g = np.array([complex(gamma).real, complex(gamma).imag])
    reason = ctypes.c_int32(0)
    steps, rej, newt = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    tend = ctypes.c_double(0.0)
    co = _copts(opts)
    st = lib().ora_track_path(L, ctypes.byref(co), s.n_eq, s.n_var, *[_p(a) for a in arrs],
                              1 if start is not None else 0, *[_p(a) for a in garrs], _p(g),
                              _p(x), ctypes.byref(reason), ctypes.byref(steps), ctypes.byref(rej),
                              ctypes.byref(newt), ctypes.byref(tend))
    return dict(x=x, status=int(st), reason=int(reason.value), steps=int(steps.value),
                rejected=int(rej.value), newton=int(newt.value), t=float(tend.value))


def track(s, gamma, paths, opts: Opts, threads: int = 1, start=None, x0=None):
    """Track paths of gamma(1-t) g + t f.  With ``start`` None, ``paths`` lists
    start-solution indices of the total-degree start system (roots of unity);
    with a start system g, ``x0`` [npaths, n, 2, L] holds its start points and
    ``paths`` only counts them.  Returns x [npaths, n, 2, L], status, reason,
    steps, newton arrays."""
    L = opts.prec
    deg = degrees(s)
    paths = np.asarray(paths, dtype=np.int64)
    npaths = len(paths)
    if start is not None:
        assert x0 is not None and len(x0) == npaths
    X = np.zeros((npaths, s.n_var, 2, L))
    status = np.zeros(npaths, dtype=np.int8)
    reason = np.zeros(npaths, dtype=np.int8)
    steps = np.zeros(npaths, dtype=np.int64)
    newton = np.zeros(npaths, dtype=np.int64)

    def work(k):
        xs = x0[k] if x0 is not None else start_solution(L, deg, int(paths[k]))
        r = track_path(s, gamma, xs, opts, start=start)
        X[k] = r["x"]
        status[k] = r["status"]
        reason[k] = r["reason"]
        steps[k] = r["steps"]
        newton[k] = r["newton"]

    if threads <= 1:
        for k in range(npaths):
            work(k)
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(work, range(npaths)))
    return dict(x=X, status=status, reason=reason, steps=steps, newton=newton)
