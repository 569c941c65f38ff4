"""GPU parity of ph_track / ph_track_batch against the oracle's tracker.

Endpoint parity: ||x_gpu - x_ref||_inf / max(1, ||x_ref||_inf) <= 1e-8
after polishing, where x_ref is the oracle's PLAIN track at the same precision.
When the two disagree on a path, the oracle re-tracks it with h_max / 10; the GPU
endpoint must then agree with the re-track (the other one jumped paths).
The step sequence is pinned on f = g only (its hand-derived count); elsewhere
step counts are compared statistically.
"""
import os

import numpy as np
import pytest

import oracle
import paper_1505_00383_amd as ph
from paper_1505_00383_amd import synth

pytestmark = pytest.mark.gpu
THREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _x_end(res, n, L, npaths):
    return ph.from_soa(res["x_end"], npaths, (n, 2, L))


def _rel(a, b):
    """per path ||a - b||_inf / max(1, ||b||_inf) on [p, n, 2, L] limb arrays."""
    d = np.abs((a - b).sum(-1)).max(-1).max(-1)
    nb = np.abs(b.sum(-1)).max(-1).max(-1)
    return d / np.maximum(1.0, nb)


def _member(res, k, n, L):
    """The results of batch member k as a single-homotopy result."""
    a, b = int(res["path_off"][k]), int(res["path_off"][k + 1])
    return {"x_end": res["x_end"][:n * 2 * L, a:b], "status": res["status"][a:b],
            "steps": res["steps"][a:b]}


def _parity(sysm, gamma, L, res, paths, oracle_mixed=0, note="", order=1, start=None, x0=None):
    """Compare GPU endpoints and verdicts with the oracle's plain track, path by
    path.  Where the two disagree (an endpoint beyond 1e-8, or a different
    status), the oracle re-tracks that path with ten times smaller steps; the
    GPU must agree with the re-track (same status and, on success, the same
    endpoint): the other side jumped paths or took a fragile decision."""
    npaths = len(paths)
    xg = _x_end(res, sysm.n_var, L, npaths)
    ref = oracle.track(sysm, gamma, paths, oracle.Opts(prec=L, mixed=oracle_mixed, predictor_order=order),
                       threads=THREADS, start=start, x0=x0)
    both_ok = (res["status"] == 1) & (ref["status"] == 1)
    rel = _rel(xg, ref["x"])
    bad = np.where((both_ok & (rel > 1e-8)) | (res["status"] != ref["status"]))[0]
    for b in bad:
        fine = oracle.track(sysm, gamma, paths[b:b + 1],
                            oracle.Opts(prec=L, mixed=oracle_mixed, h_max=0.01, h_init=0.001,
                                        predictor_order=order),
                            start=start, x0=None if x0 is None else x0[b:b + 1])
        assert fine["status"][0] == res["status"][b], (note, int(paths[b]), res["status"][b],
                                                        ref["status"][b], fine["status"][0])
        if fine["status"][0] == 1:
            r2 = _rel(xg[b:b + 1], fine["x"])[0]
            assert r2 <= 1e-8, (note, int(paths[b]), rel[b], r2)
    gs, os_ = res["steps"].astype(float), ref["steps"].astype(float)
    print(f"[gpu] {note} L={L} paths={npaths} success gpu={np.sum(res['status'] == 1)} "
          f"oracle={np.sum(ref['status'] == 1)} arbitrated={len(bad)} "
          f"max_rel={rel[both_ok].max() if both_ok.any() else 0:.2e} "
          f"mean_steps gpu={gs.mean():.1f} oracle={os_.mean():.1f}", flush=True)
    return ref, rel


@pytest.mark.parametrize("L,mixed", [(1, 0), (2, 0), (2, 1), (4, 0), (4, 1)])
def test_track_small_system(L, mixed):
    s = synth.tracking_small()
    g = synth.gamma_of(s)
    S = ph.System(s)
    res = ph.track(S, g, 8, ph.track_opts(prec=L, mixed=mixed))
    assert np.all(res["status"] == 1)
    ref, rel = _parity(s, g, L, res, np.arange(8), note=f"n3 mixed={mixed}")
    assert np.all(rel <= 1e-8)
    if L == 1:
        # same arithmetic decisions in double: identical step counts expected
        assert np.mean(np.abs(res["steps"] - ref["steps"])) <= 0.1 * np.mean(ref["steps"])
    rep = res["report"]
    assert rep["n_success"] == 8 and rep["n_fail"] == 0 and rep["steps"] == int(res["steps"].sum())


@pytest.mark.parametrize("mixed", [1, 0])
def test_track_cubic_subset_double_double(mixed):
    s = synth.tracking_cubic()
    g = synth.gamma_of(s)
    S = ph.System(s)
    paths = np.arange(48) * 131 % 6561
    xs = ph.start_solutions(S, 2, 0, 6561)
    import torch
    x0 = xs[:, torch.as_tensor(paths, device="cuda")].contiguous()
    res = ph.track(S, g, len(paths), ph.track_opts(prec=2, mixed=mixed), x_start=x0)
    _parity(s, g, 2, res, paths, note=f"n8 d3 mixed={mixed}")


def test_track_quadratic16_subset_quad_double_mixed():
    s = synth.tracking_quadratic16()
    g = synth.gamma_of(s)
    S = ph.System(s)
    npaths = 16
    res = ph.track(S, g, npaths, ph.track_opts(prec=4, mixed=1))
    _parity(s, g, 4, res, np.arange(npaths), note="n16 d2 QD mixed")


def test_bezout_count_cubic_all_paths_gpu():
    """All 3^8 = 6561 paths of the degree-3 system in double double (mixed):
    every path succeeds, the 6561 endpoints are pairwise distinct and their
    residual |f(x)| is at the rounding level."""
    import torch
    s = synth.tracking_cubic()
    g = synth.gamma_of(s)
    S = ph.System(s)
    B = 3 ** 8
    res = ph.track(S, g, B, ph.track_opts(prec=2, mixed=1))
    print(f"[gpu] bezout n8 d3: {res['report']}", flush=True)
    assert np.sum(res["status"] == 1) == B
    X = _x_end(res, 8, 2, B)
    Z = X[..., 0, 0] + 1j * X[..., 1, 0]
    key = np.round(Z / 1e-6)
    uniq = np.unique(np.concatenate([key.real, key.imag], axis=1), axis=0)
    assert len(uniq) == B
    # residual at the endpoints with the (parity-tested) GPU evaluation, t = 1
    val, _ = ph.eval_jac(S, res["x_end"], B, 2, None, g, want_jac=False)
    torch.cuda.synchronize()
    V = ph.from_soa(val, B, (8, 2, 2)).sum(-1)
    mag = 1.0 + np.abs(Z).max(axis=1) ** 3
    assert np.max(np.abs(V).max(-1).max(-1) / mag) <= 1e-26


def test_schedule_independence_bitwise():
    """The same paths give bitwise identical endpoints, status and step counts
    whatever the number of persistent workgroups (per-path work never reads
    another path's lanes)."""
    s = synth.tracking_cubic()
    g = synth.gamma_of(s)
    S = ph.System(s)
    outs = []
    for cap in ("1", "7", ""):
        if cap:
            os.environ["PH_TRACK_BLOCKS"] = cap
        else:
            os.environ.pop("PH_TRACK_BLOCKS", None)
        r = ph.track(S, g, 300, ph.track_opts(prec=2, mixed=1))
        outs.append((r["x_end"].cpu().numpy(), r["status"], r["steps"], r["reason"]))
    os.environ.pop("PH_TRACK_BLOCKS", None)
    for o in outs[1:]:
        for u, v in zip(outs[0], o):
            assert np.array_equal(u, v)


def test_forced_failures_gpu():
    import torch
    # one finite root, one path to infinity
    f = synth.system_from_terms(1, [[(0.0, {0: 2}), (1.0, {0: 1}), (-1.0, {})]])
    g = complex(np.cos(0.7), np.sin(0.7))
    r = ph.track(ph.System(f), g, 2, ph.track_opts())
    assert sorted(ph.REASONS[int(v)] for v in r["reason"]) == ["DIVERGED", "SUCCESS"]
    s = synth.tracking_small()
    gs = synth.gamma_of(s)
    S = ph.System(s)
    x0 = ph.start_solutions(S, 1, 0, 4)
    x0[1, 2] = float("nan")           # path 2 starts at NaN
    r = ph.track(S, gs, 4, ph.track_opts(), x_start=x0)
    assert ph.REASONS[int(r["reason"][2])] == "NAN" and r["status"][2] == -1
    assert np.all(r["status"][[0, 1, 3]] == 1)
    r = ph.track(S, gs, 2, ph.track_opts(h_min=0.1, h_init=0.01))
    assert all(ph.REASONS[int(v)] == "STEP_UNDERFLOW" for v in r["reason"])
    r = ph.track(S, gs, 2, ph.track_opts(max_steps=1))
    assert all(ph.REASONS[int(v)] == "MAX_STEPS" for v in r["reason"])
    sq = synth.system_from_terms(2, [[(1, {0: 2}), (-1, {})], [(1, {1: 2}), (-1, {})]])
    z = torch.zeros((4, 1), dtype=torch.float64, device="cuda")
    r = ph.track(ph.System(sq), gs, 1, ph.track_opts(), x_start=z)
    assert ph.REASONS[int(r["reason"][0])] == "SINGULAR"
    assert r["report"]["n_singular"] == 1


def test_batch_heterogeneous_small():
    """Three systems of different n in one launch, against the oracle per system."""
    rng = np.random.default_rng(3)
    systems, gammas = [], []
    for n, d in ((3, 2), (5, 2), (4, 3)):
        eqs = [synth._equation_with_anchor(rng, list(range(n)), i, d, 6) for i in range(n)]
        systems.append(synth.system_from_terms(n, eqs))
        gammas.append(synth.unit_complex(rng))
    paths = [np.arange(8), np.array([0, 5, 17, 31]), np.array([1, 40, 80])]
    res = ph.track_batch([ph.System(s) for s in systems], gammas, paths, ph.track_opts(prec=2, mixed=1))
    off = res["path_off"]
    for k, s in enumerate(systems):
        _parity(s, gammas[k], 2, _member(res, k, s.n_var, 2), paths[k], note=f"batch member {k}")


def test_graph_schedule_matches_persistent_bitwise():
    """The round kernel replayed from a captured hipGraph (slot state kept in
    device memory between launches, only the active-wave count read back)
    gives bitwise the same endpoints, status and step counts as the
    persistent kernel."""
    s = synth.tracking_cubic()
    g = synth.gamma_of(s)
    S = ph.System(s)
    a = ph.track(S, g, 500, ph.track_opts(prec=2, mixed=1))
    b = ph.track(S, g, 500, ph.track_opts(prec=2, mixed=1, schedule=ph.SCHED_GRAPH,
                                          rounds_per_launch=5, launches_per_sync=3, launch_ms=0.0))
    # launches ended by a time budget (here 0.05 ms: a few rounds each)
    c = ph.track(S, g, 500, ph.track_opts(prec=2, mixed=1, schedule=ph.SCHED_GRAPH,
                                          launches_per_sync=3, launch_ms=0.05))
    print(f"[gpu] graph schedule: persistent {a['report']['seconds']:.3f}s graph "
          f"{b['report']['seconds']:.3f}s timed launches {c['report']['seconds']:.3f}s", flush=True)
    for r in (b, c):
        assert np.array_equal(a["x_end"].cpu().numpy(), r["x_end"].cpu().numpy())
        for k in ("status", "reason", "steps"):
            assert np.array_equal(a[k], r[k])
        assert a["report"]["newton_its"] == r["report"]["newton_its"]


def test_more_workgroups_asked_than_fit_a_cu():
    """16384 paths of the n = 16 system need 4096 workgroups: more than the
    CUs hold at once even at the default 8 per CU.  Asked for 64 per CU, the
    launch is capped at what the kernel fits on a CU, so every workgroup of a
    round launch starts with it; both schedules give bitwise the same
    endpoints, status and step counts as the default launch."""
    s = synth.tracking_quadratic16()
    g = synth.gamma_of(s)
    S = ph.System(s)
    base = ph.track_opts(prec=2, mixed=1)
    print("[gpu] 16384 paths, 64 workgroups per CU asked", flush=True)
    a = ph.track(S, g, 16384, base)
    b = ph.track(S, g, 16384, ph.track_opts(prec=2, mixed=1, blocks_per_cu=64))
    c = ph.track(S, g, 16384, ph.track_opts(prec=2, mixed=1, blocks_per_cu=64, schedule=ph.SCHED_GRAPH,
                                            launch_ms=1.0))
    print(f"[gpu] default {a['report']['seconds']:.3f}s persistent-64 {b['report']['seconds']:.3f}s "
          f"graph-64 {c['report']['seconds']:.3f}s", flush=True)
    assert np.sum(a["status"] == 1) > 16000
    for r in (b, c):
        assert np.array_equal(a["x_end"].cpu().numpy(), r["x_end"].cpu().numpy())
        for k in ("status", "reason", "steps"):
            assert np.array_equal(a[k], r[k])


@pytest.mark.parametrize("schedule", [0, 1])
def test_batch_lane_classes(schedule):
    """Systems of n = 3, 6, 12 (4, 8 and 16 lanes per path) in one launch."""
    rng = np.random.default_rng(17)
    systems, gammas, paths = [], [], []
    for n, nt, npath in ((3, 5, 8), (6, 7, 40), (12, 6, 24), (5, 5, 32)):
        eqs = [synth._equation_with_anchor(rng, list(range(n)), i, 2, nt) for i in range(n)]
        systems.append(synth.system_from_terms(n, eqs))
        gammas.append(synth.unit_complex(rng))
        paths.append(np.sort(rng.choice(2 ** n, size=min(npath, 2 ** n), replace=False)))
    res = ph.track_batch([ph.System(x) for x in systems], gammas, paths,
                         ph.track_opts(prec=2, mixed=1, schedule=schedule, rounds_per_launch=16,
                                       launch_ms=0.0))
    for k, sy in enumerate(systems):
        _parity(sy, gammas[k], 2, _member(res, k, sy.n_var, 2), paths[k],
                note=f"class batch n={sy.n_var} schedule={schedule}")


def test_batch_shared_sweeps_bitwise():
    """A batch of systems with n = 3, 6, 12 and 5 (4, 8, 16 and 8 natural
    lanes) under 32 lanes per path, where eight, four, two and four lanes
    share each equation's term sweeps, against 16 lanes per path (four, two,
    one and two): endpoints, status and step counts bitwise equal, under both
    schedules.  (This batch is small enough that the default doubles the
    natural counts, so the natural counts alone are not selectable here; the
    single-system test compares them.)"""
    import torch
    rng = np.random.default_rng(19)
    systems, gammas, paths = [], [], []
    for n, nt, npath in ((3, 5, 8), (6, 7, 40), (12, 6, 24), (5, 5, 32)):
        eqs = [synth._equation_with_anchor(rng, list(range(n)), i, 2, nt) for i in range(n)]
        systems.append(synth.system_from_terms(n, eqs))
        gammas.append(synth.unit_complex(rng))
        paths.append(np.sort(rng.choice(2 ** n, size=min(npath, 2 ** n), replace=False)))
    handles = [ph.System(x) for x in systems]
    for L, mixed in ((2, 1), (4, 0)):
        base = ph.track_batch(handles, gammas, paths, ph.track_opts(prec=L, mixed=mixed, lanes_per_path=16))
        for sched in (ph.SCHED_PERSISTENT, ph.SCHED_GRAPH):
            r = ph.track_batch(handles, gammas, paths,
                               ph.track_opts(prec=L, mixed=mixed, lanes_per_path=32, schedule=sched))
            assert (base["status"] == r["status"]).all() and (base["steps"] == r["steps"]).all()
            assert torch.equal(base["x_end"], r["x_end"]), (L, mixed, sched)
        assert (base["status"] == 1).mean() > 0.9


def _distinct(X, ok):
    Z = X[ok][..., 0, 0] + 1j * X[ok][..., 1, 0]
    key = np.round(Z / 1e-6)
    return len(np.unique(np.concatenate([key.real, key.imag], axis=1), axis=0)) == len(Z)


def test_quadratic16_full_65536_paths_qd_mixed():
    """The full n = 16, degree-2 workload (2^16 paths, QD residual, FP64
    Newton solves) in the launch the benchmark times: sampled endpoints
    against the oracle's plain QD track, all successful endpoints pairwise
    distinct, and the failures counted by reason."""
    s = synth.tracking_quadratic16()
    g = synth.gamma_of(s)
    S = ph.System(s)
    B = 2 ** 16
    res = ph.track(S, g, B, ph.track_opts(prec=4, mixed=1))
    rep = res["report"]
    print(f"[gpu] n16 d2 full: {rep}", flush=True)
    ok = res["status"] == 1
    assert ok.sum() >= 0.99 * B
    assert rep["n_success"] == ok.sum() and rep["n_fail"] == B - ok.sum()
    X = _x_end(res, 16, 4, B)
    assert _distinct(X, ok)
    sample = np.array([0, 1, 12345, 32768, 54321, B - 1])
    import torch
    it = torch.as_tensor(sample, device="cuda")
    sub = {"x_end": res["x_end"][:, it], "status": res["status"][sample], "steps": res["steps"][sample]}
    _parity(s, g, 4, sub, sample, note="n16 d2 QD full, sampled")


def test_batch_full_workload_graph_schedule():
    """64 systems with n in 4..16, about 200k paths, DD residual with FP64
    solves, one launch under the graph schedule: sampled paths of eight
    systems against the oracle, every fully tracked system's endpoints
    pairwise distinct, and the report consistent with the status array."""
    sysms, gammas, paths, cap = synth.batch_heterogeneous()
    systems = [ph.System(s) for s in sysms]
    opts = ph.track_opts(prec=2, mixed=1, schedule=ph.SCHED_GRAPH)
    res = ph.track_batch(systems, gammas, paths, opts)
    off = res["path_off"]
    total = int(off[-1])
    rep = res["report"]
    print(f"[gpu] batch64: paths={total} cap={cap} {rep}", flush=True)
    assert total >= 200_000
    ok = res["status"] == 1
    assert rep["n_success"] == ok.sum() and ok.mean() >= 0.99
    X = _x_end(res, 16, 2, total)
    for k, s in enumerate(sysms):
        sl = slice(off[k], off[k + 1])
        bez = int(np.prod(s.degrees().astype(np.int64)))
        if len(paths[k]) == bez and ok[sl].all():
            assert _distinct(X[sl, :s.n_var], ok[sl]), k
    rng = np.random.default_rng(17)
    for k in rng.choice(len(sysms), size=8, replace=False):
        s = sysms[k]
        j = int(rng.integers(0, len(paths[k])))
        gi = int(off[k]) + j
        sub = {"x_end": res["x_end"][:s.n_var * 2 * 2, gi:gi + 1], "status": res["status"][gi:gi + 1],
               "steps": res["steps"][gi:gi + 1]}
        _parity(s, gammas[k], 2, sub, paths[k][j:j + 1], note=f"batch64 system {int(k)}")


@pytest.mark.parametrize("L,mixed", [(1, 0), (2, 0), (2, 1), (4, 1)])
def test_track_small_system_order4(L, mixed):
    """Fourth-order predictor (current and four previous points): endpoints
    against the oracle's order-4 track; in double the same decisions give the
    same step counts."""
    s = synth.tracking_small()
    g = synth.gamma_of(s)
    S = ph.System(s)
    res = ph.track(S, g, 8, ph.track_opts(prec=L, mixed=mixed, predictor_order=4))
    assert np.all(res["status"] == 1)
    ref, rel = _parity(s, g, L, res, np.arange(8), note=f"n3 order4 mixed={mixed}", order=4)
    assert np.all(rel <= 1e-8)
    if L == 1:
        assert np.mean(np.abs(res["steps"] - ref["steps"])) <= 0.1 * np.mean(ref["steps"])


@pytest.mark.parametrize("order", [2, 3, 4])
def test_track_cubic_subset_higher_order(order):
    s = synth.tracking_cubic()
    g = synth.gamma_of(s)
    S = ph.System(s)
    paths = np.arange(40) * 157 % 6561
    import torch
    x0 = ph.start_solutions(S, 2, 0, 6561)[:, torch.as_tensor(paths, device="cuda")].contiguous()
    res = ph.track(S, g, len(paths), ph.track_opts(prec=2, mixed=1, predictor_order=order), x_start=x0)
    _parity(s, g, 2, res, paths, note=f"n8 d3 DD mixed order {order}", order=order)


def test_track_quadratic16_subset_order4_qd_mixed():
    s = synth.tracking_quadratic16()
    g = synth.gamma_of(s)
    S = ph.System(s)
    res = ph.track(S, g, 16, ph.track_opts(prec=4, mixed=1, predictor_order=4))
    _parity(s, g, 4, res, np.arange(16), note="n16 d2 QD mixed order 4", order=4)


def test_order4_graph_schedule_matches_persistent_bitwise():
    """The predictor history lives in device memory per lane slot: replaying
    the round kernel from a graph gives bitwise the persistent results."""
    s = synth.tracking_cubic()
    g = synth.gamma_of(s)
    S = ph.System(s)
    a = ph.track(S, g, 300, ph.track_opts(prec=2, mixed=1, predictor_order=4))
    b = ph.track(S, g, 300, ph.track_opts(prec=2, mixed=1, predictor_order=4, schedule=ph.SCHED_GRAPH,
                                          rounds_per_launch=3, launches_per_sync=5, launch_ms=0.0))
    import torch
    assert (a["status"] == b["status"]).all() and (a["steps"] == b["steps"]).all()
    assert torch.equal(a["x_end"], b["x_end"])
    print(f"[gpu] order 4: steps/path {a['steps'].mean():.1f}", flush=True)


@pytest.mark.parametrize("lanes", [16, 32])
def test_more_lanes_per_path_same_results(lanes):
    """Giving each path two or four times its natural lane count (8 for
    n = 8: the extra lanes share each equation's term sweeps and the first
    lane of an equation adds the contributions in term order) changes nothing
    in the arithmetic: endpoints, status and step counts are bitwise those of
    the natural lane count, in double-double and quad-double residuals."""
    s = synth.tracking_cubic()
    g = synth.gamma_of(s)
    S = ph.System(s)
    a = ph.track(S, g, 400, ph.track_opts(prec=2, mixed=1, lanes_per_path=8))
    b = ph.track(S, g, 400, ph.track_opts(prec=2, mixed=1, lanes_per_path=lanes))
    import torch
    assert (a["status"] == b["status"]).all() and (a["steps"] == b["steps"]).all()
    assert torch.equal(a["x_end"], b["x_end"])
    # quad-double plain (the hand-over carries four limbs per partial)
    paths = np.arange(0, 6561, 97)
    x0 = ph.start_solutions(S, 4, 0, 6561)[:, torch.as_tensor(paths, device="cuda")].contiguous()
    c = ph.track(S, g, len(paths), ph.track_opts(prec=4, mixed=0, lanes_per_path=8), x_start=x0)
    d = ph.track(S, g, len(paths), ph.track_opts(prec=4, mixed=0, lanes_per_path=lanes), x_start=x0)
    assert (c["status"] == d["status"]).all() and (c["steps"] == d["steps"]).all()
    assert torch.equal(c["x_end"], d["x_end"])
    # and the default on a few paths takes the doubled count: the same results
    e = ph.track(S, g, 400, ph.track_opts(prec=2, mixed=1))
    assert torch.equal(a["x_end"], e["x_end"]) and (a["steps"] == e["steps"]).all()


def test_empty_inputs_and_empty_batch_member():
    """No paths at all returns at once with an empty report; a batch member
    with no paths between two others changes nothing for them."""
    s = synth.tracking_small()
    g = synth.gamma_of(s)
    S = ph.System(s)
    r0 = ph.track(S, g, 0, ph.track_opts(prec=2, mixed=1))
    assert r0["report"]["n_success"] == 0 and r0["report"]["steps"] == 0
    cub = synth.tracking_cubic()
    C = ph.System(cub)
    gc = synth.gamma_of(cub)
    paths = [np.arange(8), np.array([], dtype=np.int64), np.arange(1, 8, 2)]
    res = ph.track_batch([S, C, S], [g, gc, g], paths, ph.track_opts(prec=2, mixed=1))
    off = res["path_off"]
    assert list(off) == [0, 8, 8, 12]
    with pytest.raises(ph.PHError, match="-1"):
        ph.track_batch([S], [g], [np.array([3, 8])], ph.track_opts(prec=2, mixed=1))
    alone = ph.track(S, g, 8, ph.track_opts(prec=2, mixed=1))
    X = ph.from_soa(res["x_end"], 12, (8, 2, 2))
    Xa = ph.from_soa(alone["x_end"], 8, (3, 2, 2))
    assert np.all(res["status"] == 1)
    assert np.array_equal(X[:8, :3], Xa) and np.array_equal(res["steps"][:8], alone["steps"])


@pytest.mark.parametrize("L,mixed", [(1, 0), (2, 0), (2, 1), (4, 1)])
def test_track_custom_start_system(L, mixed):
    """ph_track from an explicit start system g (Eq. (1) allows any g with
    known roots): g_i = a_i x_i^2 - b_i with random complex a_i, b_i, its roots
    as start points, against the oracle tracking the same homotopy."""
    from tests.starts import diagonal_roots, diagonal_start
    s = synth.tracking_small()
    gam = synth.gamma_of(s)
    gsys, a, b = diagonal_start(np.random.default_rng(41), [2, 2, 2])
    paths = np.arange(8)
    X0 = diagonal_roots(a, b, [2, 2, 2], L, paths)
    S, G = ph.System(s), ph.System(gsys)
    res = ph.track(S, gam, 8, ph.track_opts(prec=L, mixed=mixed), x_start=ph.to_soa(X0), start=G)
    assert np.all(res["status"] == 1)
    _parity(s, gam, L, res, paths, note=f"custom start mixed={mixed}", start=gsys, x0=X0)


def test_track_quad_double_degree_three_subset():
    """QD residual with FP64 solves on the n = 8, degree-3 workload, whose start
    points include the roots exp(+-2 pi i / 3) with sqrt(3)/2 in four limbs."""
    s = synth.tracking_cubic()
    g = synth.gamma_of(s)
    S = ph.System(s)
    paths = np.array([0, 1, 2, 5, 13, 40, 121, 364, 1093, 3280, 4000, 6560])
    import torch
    x0 = ph.start_solutions(S, 4, 0, 6561)[:, torch.as_tensor(paths, device="cuda")].contiguous()
    res = ph.track(S, g, len(paths), ph.track_opts(prec=4, mixed=1), x_start=x0)
    _parity(s, g, 4, res, paths, note="n8 d3 QD mixed")


def test_residual_test_and_endpoint_check_on_gpu():
    """The residual half of the convergence test and the check of the polished
    endpoint, as in the oracle's pins: a residual tolerance no point can meet
    ends every path by step underflow; a loose corrector that accepts x = 1.75
    at t = 1 for f = -(x - 2)(x - 4) is polished to x = 2, which fails the
    path as DIVERGED under diverge_norm = 1.9 and succeeds without it."""
    s = synth.tracking_small()
    r = ph.track(ph.System(s), synth.gamma_of(s), 4, ph.track_opts(tol_res=1e-300))
    assert all(ph.REASONS[int(v)] == "STEP_UNDERFLOW" for v in r["reason"])
    f = synth.system_from_terms(1, [[(-1, {0: 2}), (6, {0: 1}), (-8, {})]])
    F = ph.System(f)
    gamma = complex(np.cos(0.3), np.sin(0.3))
    loose = dict(prec=1, tol_dx=0.5, tol_res=float("inf"), h_init=1.0, h_max=1.0, max_newton=1)
    r1 = ph.track(F, gamma, 1, ph.track_opts(**loose))
    assert r1["status"][0] == 1 and r1["steps"][0] == 1
    assert abs(ph.from_soa(r1["x_end"], 1, (1, 2, 1))[0, 0, 0, 0] - 2.0) <= 1e-14
    r2 = ph.track(F, gamma, 1, ph.track_opts(**loose, diverge_norm=1.9))
    assert r2["status"][0] == -1 and ph.REASONS[int(r2["reason"][0])] == "DIVERGED"


@pytest.mark.parametrize("L,mixed", [(1, 0), (2, 1), (4, 0)])
def test_f_equals_g_step_sequence_by_hand_gpu(L, mixed):
    """f = g: every path stays at its start point, every step is accepted
    with one Newton step, and the step count is the hand-derived one of
    tests/golden/step_sequence_f_equals_g.txt on both schedules."""
    want = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "step_sequence_f_equals_g.txt")) as f:
        for ln in f:
            if ln.strip() and not ln.startswith("#"):
                k, v = ln.split()
                want[k] = int(v)
    n, deg = 3, [2, 3, 2]
    s = synth.system_from_terms(n, [[(1, {i: deg[i]}), (-1, {})] for i in range(n)])
    gamma = complex(np.cos(1.1), np.sin(1.1))
    S = ph.System(s)
    for sched in (ph.SCHED_PERSISTENT, ph.SCHED_GRAPH):
        print(f"[gpu] f = g step count L={L} mixed={mixed} schedule={sched}", flush=True)
        res = ph.track(S, gamma, 12, ph.track_opts(prec=L, mixed=mixed, schedule=sched))
        assert np.all(res["status"] == 1)
        assert np.all(res["steps"] == want["steps"]), res["steps"]
        assert res["report"]["rejected"] == 0
        assert res["report"]["newton_its"] == 12 * want["newton"]
        x = _x_end(res, n, L, 12)
        for p in range(12):
            x0 = oracle.start_solution(L, np.array(deg, dtype=np.int32), p)
            assert np.max(np.abs(x[p].sum(-1) - np.asarray(x0).reshape(n, 2, L).sum(-1))) <= 1e-14
