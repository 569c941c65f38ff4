"""Python binding of libph (many-path polynomial homotopy hot path on MI355X).

Argument marshalling only: every step of evaluation and tracking runs in the
HIP kernels of ``libph.so``; torch provides device memory and streams.  The
library is loaded lazily and any call fails loudly (``PHError``) when it is
missing or no GPU is present -- there is no CPU fallback.

Layouts (see include/ph.h): point data is structure-of-arrays with the point
index fastest.  ``to_soa`` / ``from_soa`` convert between the natural
[npts, n, 2, L] array and the [n*2*L, ld] device matrix.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libph.so")

PH_D, PH_DD, PH_QD = 1, 2, 4
REASONS = {0: "NONE", 1: "SUCCESS", 2: "DIVERGED", 3: "STEP_UNDERFLOW", 4: "MAX_STEPS",
           5: "SINGULAR", 6: "NAN"}
EXPORTED = ["ph_system_create", "ph_system_destroy", "ph_system_info", "ph_system_degrees",
            "ph_start_solutions", "ph_eval_jac", "ph_track_opts_default", "ph_last_error",
            "ph_arith_probe", "ph_track", "ph_track_batch", "ph_eval_set_config",
            "ph_eval_autotune", "ph_track_autotune", "ph_eval_get_config", "ph_eval_prepare",
            "ph_track_noalloc"]

# ph_eval_set_config kernels
EVAL_AUTO, EVAL_GENERAL, EVAL_REGROW, EVAL_FAST, EVAL_FAST_VECROW, EVAL_UNFUSED = 0, 1, 2, 3, 4, 5


class TrackOpts(ctypes.Structure):
    """Mirror of ph_track_opts (include/ph.h)."""
    _fields_ = [("prec", ctypes.c_int32), ("mixed", ctypes.c_int32),
                ("predictor_order", ctypes.c_int32), ("max_newton", ctypes.c_int32),
                ("expand_after", ctypes.c_int32), ("polish_max", ctypes.c_int32),
                ("h_init", ctypes.c_double), ("h_min", ctypes.c_double),
                ("h_max", ctypes.c_double), ("shrink", ctypes.c_double),
                ("expand", ctypes.c_double), ("tol_dx", ctypes.c_double),
                ("diverge_norm", ctypes.c_double), ("polish_tol", ctypes.c_double),
                ("max_steps", ctypes.c_int64), ("schedule", ctypes.c_int32),
                ("rounds_per_launch", ctypes.c_int32), ("launches_per_sync", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("lanes_per_path", ctypes.c_int32),
                ("tol_res", ctypes.c_double), ("launch_ms", ctypes.c_double)]


SCHED_PERSISTENT, SCHED_GRAPH = 0, 1


class TrackReport(ctypes.Structure):
    """Mirror of ph_track_report."""
    _fields_ = [(n, ctypes.c_int64) for n in ("n_success", "n_fail", "n_diverged",
                                               "n_step_underflow", "n_max_steps", "n_singular",
                                               "n_nan", "steps", "rejected", "newton_its")] + \
               [("seconds", ctypes.c_double)]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


def track_opts(**kw) -> TrackOpts:
    """ph_track_opts_default() with keyword overrides."""
    o = TrackOpts()
    _check(load_library().ph_track_opts_default(ctypes.byref(o)))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


class PHError(RuntimeError):
    pass


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libph.so (no GPU needed for loading).  Raises PHError if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise PHError(f"{path} is missing: build it with `python -m paper_1505_00383_amd.build`")
    L = ctypes.CDLL(path)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.ph_system_create.argtypes = [i32, i32, P, P, P, P, P, i32, ctypes.POINTER(P)]
    L.ph_system_destroy.argtypes = [P]
    L.ph_system_info.argtypes = [P, P, P, P, P]
    L.ph_system_degrees.argtypes = [P, P]
    L.ph_start_solutions.argtypes = [P, i32, i64, i64, P, i64, P]
    L.ph_eval_jac.argtypes = [P, P, P, i32, i64, P, P, i64, P, P, P]
    L.ph_track_opts_default.argtypes = [P]
    L.ph_last_error.restype = ctypes.c_char_p
    L.ph_arith_probe.argtypes = [i32, i32, i64, P, P, P, P]
    L.ph_track.argtypes = [P, P, P, i64, P, i64, P, P, P, P, P, P, P]
    L.ph_track_noalloc.argtypes = [P, P, P, i64, P, i64, P, P, P, P, P, P, P]
    L.ph_track_batch.argtypes = [i32, P, P, P, P, P, P, i64, P, P, P, P, P]
    L.ph_eval_set_config.argtypes = [P, P, i32, i32, i32, i32]
    L.ph_eval_prepare.argtypes = [P, P, i32, i64]
    L.ph_eval_get_config.argtypes = [P, P, i32, P, P, P]
    L.ph_eval_autotune.argtypes = [P, P, P, i32, i64, P, P, i64, P, P, P, P]
    L.ph_track_autotune.argtypes = [i32, P, P, P, P, P, i64, P, P, P]
    for name in EXPORTED:
        fn = getattr(L, name)
        if name != "ph_last_error":
            fn.restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != 0:
        raise PHError(f"libph error {rc}: {load_library().ph_last_error().decode()}")


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise PHError("no HIP device available: libph runs on the GPU only")
    return torch


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


# ---------------------------------------------------------------------------
# layout marshalling
# ---------------------------------------------------------------------------
def to_soa(x, ld: int | None = None, device="cuda"):
    """[npts, n, 2, L] (numpy or torch) -> device tensor [n*2*L, ld], point fastest."""
    torch = _torch()
    xt = torch.as_tensor(np.ascontiguousarray(x) if isinstance(x, np.ndarray) else x,
                         dtype=torch.float64)
    npts = xt.shape[0]
    ld = ld or npts
    rows = xt[0].numel() if npts else int(np.prod(xt.shape[1:]))
    out = torch.zeros((rows, ld), dtype=torch.float64, device=device)
    if npts:
        out[:, :npts] = xt.reshape(npts, rows).to(device).T
    return out


def from_soa(m, npts: int, shape_tail):
    """device tensor [rows, ld] -> numpy [npts, *shape_tail]."""
    return m[:, :npts].T.contiguous().cpu().numpy().reshape((npts,) + tuple(shape_tail))


# ---------------------------------------------------------------------------
# systems
# ---------------------------------------------------------------------------
class System:
    """Device term tables of a polynomial system (ph_system_create)."""

    def __init__(self, sysm, coef_limbs: int = 1):
        lib = load_library()
        self.n_eq, self.n_var = int(sysm.n_eq), int(sysm.n_var)
        eq = np.ascontiguousarray(sysm.eq_term_off, dtype=np.int32)
        tf = np.ascontiguousarray(sysm.term_fac_off, dtype=np.int32)
        fv = np.ascontiguousarray(sysm.fac_var, dtype=np.int32)
        fe = np.ascontiguousarray(sysm.fac_exp, dtype=np.int32)
        cf = np.ascontiguousarray(sysm.coef, dtype=np.float64)
        if coef_limbs != 1:
            cf = np.ascontiguousarray(cf.reshape(-1, 2, coef_limbs))
        h = ctypes.c_void_p()
        _check(lib.ph_system_create(self.n_eq, self.n_var, eq.ctypes.data, tf.ctypes.data,
                                    fv.ctypes.data if fv.size else None,
                                    fe.ctypes.data if fe.size else None, cf.ctypes.data,
                                    coef_limbs, ctypes.byref(h)))
        self._h = h
        self.source = sysm

    @property
    def handle(self):
        return self._h

    def degrees(self) -> np.ndarray:
        d = np.zeros(self.n_eq, dtype=np.int32)
        _check(load_library().ph_system_degrees(self._h, d.ctypes.data))
        return d

    def info(self):
        ne, nv, mk = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        nt = ctypes.c_int64()
        _check(load_library().ph_system_info(self._h, ctypes.byref(ne), ctypes.byref(nv), ctypes.byref(nt),
                                   ctypes.byref(mk)))
        return dict(n_eq=ne.value, n_var=nv.value, n_terms=nt.value, max_factors=mk.value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().ph_system_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def eval_jac(sys: System, x_soa, npts: int, prec: int, t=None, gamma=1.0 + 0j, start=None,
             val=None, jac=None, want_jac: bool = True, stream=None):
    """H(x,t) = gamma(1-t) g + t f and dH/dx at npts points (ph_eval_jac).

    x_soa: device [n_var*2*prec, ld]; t: device [npts] or None (t = 1).
    Returns (val [n_eq*2*prec, ld], jac [n_eq*n_var*2*prec, ld] or None)."""
    torch = _torch()
    ld = x_soa.shape[1]
    if val is None:
        val = torch.empty((sys.n_eq * 2 * prec, ld), dtype=torch.float64, device=x_soa.device)
    if want_jac and jac is None:
        jac = torch.empty((sys.n_eq * sys.n_var * 2 * prec, ld), dtype=torch.float64,
                          device=x_soa.device)
    g = (ctypes.c_double * 2)(complex(gamma).real, complex(gamma).imag)
    _check(load_library().ph_eval_jac(sys.handle, None if start is None else start.handle, g, prec, npts,
                            _ptr(t), _ptr(x_soa), ld, _ptr(val), _ptr(jac) if want_jac else None,
                            _stream(stream)))
    return val, (jac if want_jac else None)


def eval_prepare(sys: System, prec: int = 1, start: System | None = None,
                 unfused_points: int = 0):
    """Build the term tables of (sys, start) and, with unfused_points > 0, size the
    unfused design's arrays for that many points of prec limbs (ph_eval_prepare).
    ph_eval_jac itself never allocates: a start system must be prepared first."""
    _check(load_library().ph_eval_prepare(sys.handle, None if start is None else start.handle,
                                          prec, unfused_points))


def eval_set_config(sys: System, prec: int, kernel: int = EVAL_AUTO, waves: int = 0,
                    groups: int = 0, start: System | None = None):
    """Pin ph_eval_jac's kernel and tiling for (sys, start, prec) (ph_eval_set_config);
    all zero restores the automatic choice."""
    _check(load_library().ph_eval_set_config(sys.handle, None if start is None else start.handle,
                                             prec, kernel, waves, groups))


def eval_get_config(sys: System, prec: int, start: System | None = None):
    """(kernel, waves, groups) pinned or tuned for (sys, start, prec); zeros: automatic."""
    k, w, g = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(load_library().ph_eval_get_config(sys.handle, None if start is None else start.handle, prec,
                                             ctypes.byref(k), ctypes.byref(w), ctypes.byref(g)))
    return k.value, w.value, g.value


def eval_autotune(sys: System, x_soa, npts: int, prec: int, t=None, gamma=1.0 + 0j,
                  start=None, val=None, jac=None, stream=None) -> float:
    """Time every applicable kernel/tiling of ph_eval_jac on these buffers and keep
    the fastest for (sys, start, prec) (ph_eval_autotune).  Returns its ms."""
    torch = _torch()
    ld = x_soa.shape[1]
    if val is None:
        val = torch.empty((sys.n_eq * 2 * prec, ld), dtype=torch.float64, device=x_soa.device)
    if jac is None:
        jac = torch.empty((sys.n_eq * sys.n_var * 2 * prec, ld), dtype=torch.float64,
                          device=x_soa.device)
    g = (ctypes.c_double * 2)(complex(gamma).real, complex(gamma).imag)
    ms = ctypes.c_double(0.0)
    _check(load_library().ph_eval_autotune(sys.handle, None if start is None else start.handle, g,
                                           prec, npts, _ptr(t), _ptr(x_soa), ld, _ptr(val),
                                           _ptr(jac), _stream(stream), ctypes.byref(ms)))
    return ms.value


def start_solutions(sys: System, prec: int, first: int, npaths: int, out=None, stream=None):
    """Roots-of-unity start points (ph_start_solutions) -> device [n*2*prec, npaths]."""
    torch = _torch()
    if out is None:
        out = torch.empty((sys.n_var * 2 * prec, max(npaths, 1)), dtype=torch.float64,
                          device="cuda")
    _check(load_library().ph_start_solutions(sys.handle, prec, first, npaths, _ptr(out), out.shape[1],
                                   _stream(stream)))
    return out


def arith_probe(prec: int, op: int, a, b, stream=None):
    """Device arithmetic on [n, prec] reals (op 0..2) or [n, 2, prec] complexes (op 3..5)."""
    torch = _torch()
    at = torch.as_tensor(a, dtype=torch.float64).contiguous().cuda()
    bt = torch.as_tensor(b, dtype=torch.float64).contiguous().cuda()
    out = torch.empty_like(at)
    _check(load_library().ph_arith_probe(prec, op, at.shape[0], _ptr(at), _ptr(bt), _ptr(out),
                               _stream(stream)))
    return out.cpu().numpy()


def _track_outputs(torch, n_rows, total, ld):
    x_end = torch.zeros((n_rows, max(ld, 1)), dtype=torch.float64, device="cuda")
    status = torch.zeros(max(total, 1), dtype=torch.int8, device="cuda")
    reason = torch.zeros(max(total, 1), dtype=torch.int8, device="cuda")
    steps = torch.zeros(max(total, 1), dtype=torch.int32, device="cuda")
    return x_end, status, reason, steps


def track(sys: System, gamma, npaths: int, opts: TrackOpts | None = None, x_start=None,
          start: System | None = None, stream=None):
    """Track paths 0..npaths-1 of gamma(1-t) g + t f (ph_track).  x_start: device SoA
    start points [n*2*prec, ld] or None (roots of unity).  Returns a dict with
    device x_end [n*2*prec, ld] and numpy status / reason / steps, plus the report."""
    return _track_one("ph_track", sys, gamma, npaths, opts, x_start, start, stream)


def track_noalloc(sys: System, gamma, npaths: int, opts: TrackOpts | None = None, x_start=None,
                  start: System | None = None, stream=None):
    """track() through ph_track_noalloc: the library's fixed device scratch
    instead of per-call allocations (persistent schedule only; an explicit
    start system must be prepared with eval_prepare first)."""
    return _track_one("ph_track_noalloc", sys, gamma, npaths, opts, x_start, start, stream)


def _track_one(entry, sys, gamma, npaths, opts, x_start, start, stream):
    torch = _torch()
    opts = opts or track_opts()
    L = opts.prec
    ld = x_start.shape[1] if x_start is not None else max(npaths, 1)
    x_end, status, reason, steps = _track_outputs(torch, sys.n_var * 2 * L, npaths, ld)
    rep = TrackReport()
    g = (ctypes.c_double * 2)(complex(gamma).real, complex(gamma).imag)
    fn = getattr(load_library(), entry)
    _check(fn(sys.handle, None if start is None else start.handle, g, npaths, _ptr(x_start), ld,
              ctypes.byref(opts), _ptr(x_end), _ptr(status), _ptr(reason), _ptr(steps),
              ctypes.byref(rep), _stream(stream)))
    return dict(x_end=x_end, status=status[:npaths].cpu().numpy(),
                reason=reason[:npaths].cpu().numpy(), steps=steps[:npaths].cpu().numpy(),
                report=rep.as_dict())


def _batch_arrays(systems, gammas, path_lists):
    nsys = len(systems)
    counts, ids = [], []
    any_ids = any(p is not None for p in path_lists)
    for s, p in zip(systems, path_lists):
        if p is None:
            B = int(np.prod(s.degrees().astype(np.int64)))
            counts.append(B)
            if any_ids:
                ids.append(np.arange(B, dtype=np.int64))
        else:
            p = np.asarray(p, dtype=np.int64)
            counts.append(len(p))
            ids.append(p)
    off = np.zeros(nsys + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    pid = np.ascontiguousarray(np.concatenate(ids)) if any_ids else None
    handles = (ctypes.c_void_p * nsys)(*[s.handle.value for s in systems])
    gam = np.ascontiguousarray([[complex(g).real, complex(g).imag] for g in gammas],
                               dtype=np.float64)
    return nsys, handles, gam, off, pid


def track_batch(systems, gammas, path_lists, opts: TrackOpts | None = None, stream=None):
    """Track the given start-solution indices of several systems in one launch
    (ph_track_batch).  path_lists[s]: int array of multi-index numbers or None
    for every start solution of system s.  Global path order = concatenation."""
    torch = _torch()
    opts = opts or track_opts()
    L = opts.prec
    nsys, handles, gam, off, pid = _batch_arrays(systems, gammas, path_lists)
    total = int(off[-1])
    nmax = max(s.n_var for s in systems)
    x_end, status, reason, steps = _track_outputs(torch, nmax * 2 * L, total, total)
    rep = TrackReport()
    _check(load_library().ph_track_batch(nsys, handles, gam.ctypes.data, off.ctypes.data,
                                         None if pid is None else pid.ctypes.data,
                                         ctypes.byref(opts), _ptr(x_end), max(total, 1),
                                         _ptr(status), _ptr(reason), _ptr(steps),
                                         ctypes.byref(rep), _stream(stream)))
    return dict(x_end=x_end, status=status[:total].cpu().numpy(),
                reason=reason[:total].cpu().numpy(), steps=steps[:total].cpu().numpy(),
                report=rep.as_dict(), path_off=off)


def track_autotune(systems, gammas, path_lists, opts: TrackOpts | None = None,
                   sample: int = 16384, stream=None):
    """Launch shape (schedule, rounds_per_launch, blocks_per_cu, lanes_per_path) for this batch,
    timed on a proportional sample of its paths (ph_track_autotune).
    Returns (tuned TrackOpts, seconds of the sample under it; 0 from the cache)."""
    _torch()
    opts = opts or track_opts()
    nsys, handles, gam, off, pid = _batch_arrays(systems, gammas, path_lists)
    tuned = TrackOpts()
    sec = ctypes.c_double(0.0)
    _check(load_library().ph_track_autotune(nsys, handles, gam.ctypes.data, off.ctypes.data,
                                            None if pid is None else pid.ctypes.data,
                                            ctypes.byref(opts), sample, ctypes.byref(tuned),
                                            ctypes.byref(sec), _stream(stream)))
    return tuned, sec.value
