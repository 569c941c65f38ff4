"""ph_track_noalloc (the tracking entry point for callers that cannot allocate)
against ph_track: the same kernels on the same inputs, so endpoints, status,
reason and step counts must agree bit for bit.  Two calls in a row through the
library's fixed scratch, the second with a smaller input (and a different
precision and start system), check that no state of the first call leaks into
the second."""
import numpy as np
import pytest

import paper_1505_00383_amd as ph
from paper_1505_00383_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _same(a, b, npaths, rows):
    xa = a["x_end"][:rows, :npaths].cpu().numpy()
    xb = b["x_end"][:rows, :npaths].cpu().numpy()
    assert np.array_equal(xa.view(np.uint64), xb.view(np.uint64))
    for key in ("status", "reason", "steps"):
        assert np.array_equal(a[key], b[key]), key
    for key in ("n_success", "n_fail", "steps", "rejected", "newton_its"):
        assert a["report"][key] == b["report"][key], key


def test_noalloc_matches_track_two_calls_second_smaller():
    import torch
    from tests.starts import diagonal_roots, diagonal_start
    # call 1: n = 8, degree 3, DD residual with FP64 solves, fourth-order
    # predictor (history in the scratch), 2048 paths
    s = synth.tracking_cubic()
    gam = synth.gamma_of(s)
    S = ph.System(s)
    o = ph.track_opts(prec=2, mixed=1, predictor_order=4)
    print("[noalloc] call 1: n=8 d=3 DD mixed order 4, 2048 paths", flush=True)
    ref = ph.track(S, gam, 2048, o)
    got = ph.track_noalloc(S, gam, 2048, o)
    torch.cuda.synchronize()
    _same(got, ref, 2048, 8 * 2 * 2)
    assert np.sum(got["status"] == 1) > 1900
    # call 2: n = 3 from an explicit start system, QD plain, secant, 8 paths
    t = synth.tracking_small()
    gam2 = synth.gamma_of(t)
    gsys, a, b = diagonal_start(np.random.default_rng(41), [2, 2, 2])
    X0 = diagonal_roots(a, b, [2, 2, 2], 4, np.arange(8))
    T, G = ph.System(t), ph.System(gsys)
    ph.eval_prepare(T, 4, start=G)
    o2 = ph.track_opts(prec=4, mixed=0)
    print("[noalloc] call 2: n=3 QD plain, explicit start, 8 paths", flush=True)
    got2 = ph.track_noalloc(T, gam2, 8, o2, x_start=ph.to_soa(X0), start=G)
    ref2 = ph.track(T, gam2, 8, o2, x_start=ph.to_soa(X0), start=G)
    torch.cuda.synchronize()
    _same(got2, ref2, 8, 3 * 2 * 4)
    assert np.all(got2["status"] == 1)
    # call 3: the first workload again, fewer paths, after the smaller call
    print("[noalloc] call 3: n=8 d=3 DD mixed order 4, 500 paths", flush=True)
    got3 = ph.track_noalloc(S, gam, 500, o)
    torch.cuda.synchronize()
    x3 = got3["x_end"][:32, :500].cpu().numpy()
    x1 = got["x_end"][:32, :500].cpu().numpy()
    assert np.array_equal(x3.view(np.uint64), x1.view(np.uint64))
    assert np.array_equal(got3["status"], got["status"][:500])


def test_noalloc_rejections():
    s = synth.tracking_small()
    gam = synth.gamma_of(s)
    S = ph.System(s)
    o = ph.track_opts(prec=1)
    o.schedule = 1  # PH_SCHED_GRAPH
    with pytest.raises(ph.PHError, match="persistent schedule only"):
        ph.track_noalloc(S, gam, 8, o)
    # an explicit start system that was never prepared for this target
    from tests.starts import diagonal_roots, diagonal_start
    gsys, a, b = diagonal_start(np.random.default_rng(7), [2, 2, 2])
    G = ph.System(gsys)
    X0 = diagonal_roots(a, b, [2, 2, 2], 1, np.arange(8))
    with pytest.raises(ph.PHError, match="not prepared"):
        ph.track_noalloc(S, gam, 8, ph.track_opts(prec=1), x_start=ph.to_soa(X0), start=G)
    # a predictor history larger than the scratch: 65536 paths of n = 16 at
    # as many workgroups as fit the CUs (7 per CU on the MI355X: 1792
    # workgroups of 64 QD slots, 22 MB); refused before any launch
    q = synth.tracking_quadratic16()
    Q = ph.System(q)
    o3 = ph.track_opts(prec=4, mixed=1, predictor_order=4)
    o3.blocks_per_cu = 16
    with pytest.raises(ph.PHError, match="predictor history"):
        ph.track_noalloc(Q, synth.gamma_of(q), 65536, o3)
