"""Host-side pieces of bench.py: the algorithmic cost model on small terms
(counted by hand from the sweep of Table 6) and the guard that reports HBM
traffic only for the kernel sources and tiling the counters were taken with."""
import hashlib
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


class _Sys:
    """A one-equation, two-unknown system with the given term exponent lists
    (term τ uses unknowns 0..k-1)."""

    def __init__(self, terms, degs):
        self.n_var = self.n_eq = len(degs)
        self.n_terms = len(terms)
        self.fac_exp = np.array([e for t in terms for e in t], dtype=np.int32)
        off = [0]
        for t in terms:
            off.append(off[-1] + len(t))
        self.term_fac_off = np.array(off, dtype=np.int64)
        self._degs = degs

    def degrees(self):
        return np.array(self._degs)


def test_flops_per_point_counts_by_hand():
    # target term x0 x1^2 (k = 2, one exponent >= 2): 3k-3+1 = 4 products,
    # k+1 = 3 additions, 2 scalings; start terms x_i^2 (k = 1, a = 2): 1 product,
    # 2 additions, 2 scalings each; constants -1: 1 addition + 1 scaling each
    s = _Sys([[1, 2]], [2, 2])
    for L in (1, 2, 4):
        M, A, S = bench.CMUL[L], bench.CADD[L], bench.CSCALE[L]
        want = (4 * M + 3 * A + 2 * S) + 2 * (1 * M + 2 * A + 2 * S) + 2 * (A + S)
        assert bench.flops_per_point(s, L) == want


def test_bytes_per_point():
    s = _Sys([[1, 2]], [2, 2])
    # x (2 complex), H (2), J (4), t (one double)
    assert bench.bytes_per_point(s, 1) == 16 * (2 + 2 + 4) + 8
    assert bench.bytes_per_point(s, 4) == 64 * (2 + 2 + 4) + 8


def test_traffic_guard(monkeypatch):
    path = "paper_1505_00383_amd/csrc/ph_arith.hpp"
    with open(os.path.join(ROOT, path), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    table = {"k_any": {"bytes": 123, "sources": {path: sha}},
             "k_tiled": {"by_launch": {(1, 8, 4): 456, (1, 8, 1): 321}, "sources": {path: sha}},
             "k_stale": {"bytes": 789, "sources": {path: "0" * 16}}}
    monkeypatch.setattr(bench, "TRAFFIC", table)
    assert bench.traffic_of("k_any") == 123
    assert bench.traffic_of("k_any", (3, 2, 1)) == 123
    assert bench.traffic_of("k_tiled", (1, 8, 4)) == 456
    assert bench.traffic_of("k_tiled", [1, 8, 4]) == 456
    assert bench.traffic_of("k_tiled", (1, 8, 1)) == 321
    assert bench.traffic_of("k_tiled", (1, 8, 2)) is None
    assert bench.traffic_of("k_tiled") is None
    assert bench.traffic_of("k_stale") is None
    assert bench.traffic_of("unknown") is None
    # the accumulation-register kernels launch at most four waves per
    # workgroup: a larger configured count is the same launch
    monkeypatch.setattr(bench, "TRAFFIC", {"eval_dd_arow_kernel": {"by_launch": {(3, 4, 1): 7},
                                                                   "sources": {path: sha}}})
    assert bench.traffic_of("eval_dd_arow_kernel", (3, 8, 1)) == 7
    assert bench.traffic_of("eval_dd_arow_kernel", (3, 6, 1)) == 7
    assert bench.traffic_of("eval_dd_arow_kernel", (3, 2, 1)) is None


def test_mgs_flops_counts_by_hand():
    # n = 1: [J | -H] is 1 x 2; column 0: |w|^2 (1 squared modulus), r_00,
    # q = w / r (1 scaling); column 1: r_01 = q^H w_1 and the update (2
    # complex products and additions); back substitution dx = r_01 / r_00
    # (1 scaling): n^2 (n+1) = 2 products and additions, n^2 + n = 2 scalings
    for L in (1, 2, 4):
        M, A, S = bench.CMUL[L], bench.CADD[L], bench.CSCALE[L]
        assert bench.mgs_flops(1, L) == 2 * (M + A) + 2 * S + (S + A // 2)
    # the cubic growth that makes the plain QD solve dominate at n = 16
    assert bench.mgs_flops(16, 4) / bench.mgs_flops(16, 1) > 50


def test_tracker_cost_model_and_roofline():
    s = _Sys([[1, 2]], [2, 2])
    it = bench.track_iteration_flops(s, 2, 1)
    assert it == bench.flops_per_point(s, 2) + bench.mgs_flops(2, 1) + 2 * bench.CADD[2] + 4 + 8
    assert bench.track_iteration_flops(s, 2, 0) > it           # plain solves in DD
    rep = {"newton_its": 300, "steps": 100}
    r = bench.track_roofline(s, 2, 1, 1, rep, 1e-3, 10)
    want = 300 * it + 100 * bench.predictor_flops(s, 2, 1)
    assert abs(r["flops_per_path"] - want / 10) < 1e-9
    assert abs(r["fp64_frac"] - want / 1e-3 / bench.PEAK_FP64) < 1e-12


def test_limb_error_is_exact_on_cancelling_limbs():
    a = np.zeros((1, 1, 2, 2))
    b = np.zeros((1, 1, 2, 2))
    a[0, 0, 0] = [1.0, 2.0 ** -60]
    b[0, 0, 0] = [1.0, 0.0]
    assert bench._limb_err(a, b)[0] == 2.0 ** -60
    assert bench._limb_err(b, b)[0] == 0.0


def test_summary_keeps_every_cell_last():
    res = {"value": 1.0, "roofline": {"frac": 0.5},
           "extras": {"eval_prec2": {"points_per_s": 2.0, "fp64_frac": 0.4},
                      "track_n3_d2_8paths_double": {"paths_per_s": 3.0, "roofline": {"fp64_frac": 0.1},
                                                    "oracle": {"oracle_1core_paths_per_s": 5.0,
                                                               "oracle_allcores_paths_per_s": 9.0,
                                                               "oracle_allcores_threads": 2}}},
           "cpu_baseline": {"value": 7.0, "one_core_value": 1.5, "host": {"nproc": 2}}}
    out = bench.summary(res, 1)
    assert out["eval_points_per_s"] == {"D": 1.0, "DD": 2.0}
    assert out["track_paths_per_s"] == {"n3_d2_8p_D_plain": 3.0}
    assert out["oracle_track_paths_per_s"]["n3_d2_D"] == {"1core": 5.0, "allcores": 9.0, "threads": 2}
    assert out["host"] == {"nproc": 2}
    assert out["track_longest_path_alone_over_whole_run"] == {}


def test_summary_reports_the_longest_path_alone():
    run = {"paths_per_s": 4.0, "roofline": {"fp64_frac": 0.1},
           "longest_path_alone": {"path": 7, "steps": 600, "seconds": 0.9, "fraction_of_whole_run": 0.9}}
    res = {"value": 1.0, "roofline": {"frac": 0.5},
           "extras": {"track_n8_d3_6561paths": {"dd_mixed": run, "dd_plain": {"paths_per_s": 1.0}}}}
    out = bench.summary(res, 1)
    assert out["track_paths_per_s"] == {"n8_d3_6561p_DD_mixed": 4.0, "n8_d3_6561p_DD_plain": 1.0}
    assert out["track_longest_path_alone_over_whole_run"] == {"n8_d3_6561p_DD_mixed": 0.9}
