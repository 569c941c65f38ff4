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
             "k_tiled": {"bytes": 456, "launch": (1, 8, 4), "sources": {path: sha}},
             "k_stale": {"bytes": 789, "sources": {path: "0" * 16}}}
    monkeypatch.setattr(bench, "TRAFFIC", table)
    assert bench.traffic_of("k_any") == 123
    assert bench.traffic_of("k_any", (3, 2, 1)) == 123
    assert bench.traffic_of("k_tiled", (1, 8, 4)) == 456
    assert bench.traffic_of("k_tiled", [1, 8, 4]) == 456
    assert bench.traffic_of("k_tiled", (1, 8, 2)) is None
    assert bench.traffic_of("k_tiled") is None
    assert bench.traffic_of("k_stale") is None
    assert bench.traffic_of("unknown") is None
