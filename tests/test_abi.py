"""The C-ABI library loads and exports every function that include/ph.h
declares (no GPU needed), and the host-only entry points behave."""
import ctypes
import os
import re

import pytest

import paper_1505_00383_amd as ph

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "ph.h")).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(ph_\w+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ph.LIB_PATH):
        import paper_1505_00383_amd.build as b
        b.build(verbose=False)
    return ph.load_library()


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("ph_system_create", "ph_eval_jac", "ph_start_solutions", "ph_system_destroy"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_opts_default_host_only(lib):
    class Opts(ctypes.Structure):
        _fields_ = [(n, ctypes.c_int32) for n in ("prec", "mixed", "predictor_order", "max_newton",
                                                   "expand_after", "polish_max")] + \
                   [(n, ctypes.c_double) for n in ("h_init", "h_min", "h_max", "shrink", "expand",
                                                    "tol_dx", "diverge_norm", "polish_tol")] + \
                   [("max_steps", ctypes.c_int64)] + \
                   [(n, ctypes.c_int32) for n in ("schedule", "rounds_per_launch", "launches_per_sync",
                                                   "blocks_per_cu", "lanes_per_path")] + \
                   [("tol_res", ctypes.c_double), ("launch_ms", ctypes.c_double)]
    o = Opts()
    assert lib.ph_track_opts_default(ctypes.byref(o)) == 0
    assert (o.prec, o.max_newton, o.expand_after, o.polish_max) == (1, 3, 3, 8)
    assert (o.h_init, o.h_min, o.h_max, o.shrink, o.expand) == (0.01, 1e-10, 0.1, 0.5, 1.5)
    assert (o.tol_dx, o.diverge_norm, o.max_steps) == (1e-8, 1e8, 100000)
    assert (o.schedule, o.rounds_per_launch, o.launches_per_sync, o.blocks_per_cu) == (0, 32, 8, 0)
    assert o.lanes_per_path == 0 and o.tol_res == 1e-6 and o.launch_ms == 2.0
    assert ctypes.sizeof(Opts) == ctypes.sizeof(ph.TrackOpts)
    assert lib.ph_track_opts_default(None) == -1


def test_validation_errors_before_any_device_call(lib):
    import numpy as np
    h = ctypes.c_void_p()
    eq = np.array([0, 1], dtype=np.int32)
    tf = np.array([0, 1], dtype=np.int32)
    cf = np.array([1.0, 0.0])
    bad_var = np.array([5], dtype=np.int32)
    one = np.array([1], dtype=np.int32)
    rc = lib.ph_system_create(1, 1, eq.ctypes.data, tf.ctypes.data, bad_var.ctypes.data,
                              one.ctypes.data, cf.ctypes.data, 1, ctypes.byref(h))
    assert rc == -1 and b"out of range" in lib.ph_last_error()
    zero = np.array([0], dtype=np.int32)
    rc = lib.ph_system_create(1, 1, eq.ctypes.data, tf.ctypes.data, zero.ctypes.data,
                              zero.ctypes.data, cf.ctypes.data, 1, ctypes.byref(h))
    assert rc == -1 and b"exponent" in lib.ph_last_error()
    rc = lib.ph_system_create(65, 65, eq.ctypes.data, tf.ctypes.data, zero.ctypes.data,
                              one.ctypes.data, cf.ctypes.data, 1, ctypes.byref(h))
    assert rc == -4
    rc = lib.ph_system_create(1, 1, eq.ctypes.data, tf.ctypes.data, zero.ctypes.data,
                              one.ctypes.data, cf.ctypes.data, 3, ctypes.byref(h))
    assert rc == -1 and b"coef_limbs" in lib.ph_last_error()
    assert lib.ph_eval_jac(None, None, None, 1, 1, None, None, 1, None, None, None) == -1
    assert lib.ph_eval_set_config(None, None, 1, 0, 0, 0) == -1
    assert lib.ph_track_autotune(1, None, None, None, None, None, 1, None, None, None) == -1
    assert lib.ph_eval_autotune(None, None, None, 1, 1, None, None, 1, None, None, None,
                                None) == -1


def test_binding_fails_loudly_without_gpu(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    import numpy as np
    with pytest.raises(ph.PHError):
        ph.to_soa(np.zeros((1, 1, 2, 1)))
