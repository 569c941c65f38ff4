"""Kernel choice, tiling and autotuning of ph_eval_jac: every configuration
ph_eval_set_config accepts gives oracle-exact results, a kernel that does not
apply is refused, and ph_eval_autotune's choice persists in its cache file
(looked up by the systems' fingerprints)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import paper_1505_00383_amd as ph
from paper_1505_00383_amd import synth
from tests.parity import TOL, scaled_error

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _eval(S, s, L, x, t, gamma):
    import torch
    npts = x.shape[0]
    xs = ph.to_soa(x)
    tt = torch.as_tensor(np.ascontiguousarray(t), dtype=torch.float64).cuda()
    val, jm = ph.eval_jac(S, xs, npts, L, tt, gamma)
    torch.cuda.synchronize()
    return (ph.from_soa(val, npts, (s.n_eq, 2, L)),
            ph.from_soa(jm, npts, (s.n_eq, s.n_var, 2, L)))


@pytest.mark.parametrize("L", [1, 2, 4])
def test_every_configuration_matches_oracle(L):
    s = synth.eval_dense(seed=778, n=16, terms_per_eq=10, k=5)
    rng = np.random.default_rng(11)
    npts = 64 * 3 + 29
    x = synth.random_points(s.n_var, npts, L, rng, 0.95)
    t = rng.uniform(0, 1, npts)
    g = synth.gamma_of(s)
    ov, oj, sv, sj = oracle.eval_homotopy(s, L, x, t, g)
    S = ph.System(s)
    kernels = [ph.EVAL_GENERAL, ph.EVAL_UNFUSED] + ([ph.EVAL_REGROW, ph.EVAL_FAST, ph.EVAL_FAST_VECROW]
                                                   if L == 1 else [ph.EVAL_FAST])
    worst = 0.0
    ph.eval_prepare(S, L, unfused_points=npts)
    for k in kernels:
        tilings = [(0, 0)] if k == ph.EVAL_UNFUSED else [(W, G) for W in (1, 2, 4, 8) for G in (1, 2, 4)]
        for W, G in tilings:
            ph.eval_set_config(S, L, k, W, G)
            v, j = _eval(S, s, L, x, t, g)
            e = max(scaled_error(v, ov, sv), scaled_error(j, oj, sj))
            worst = max(worst, e)
            assert e <= TOL[L], (k, W, G, e)
    ph.eval_set_config(S, L)   # back to automatic
    v, j = _eval(S, s, L, x, t, g)
    assert max(scaled_error(v, ov, sv), scaled_error(j, oj, sj)) <= TOL[L]
    print(f"[gpu] L={L} configs ok, worst err/S={worst:.2e}", flush=True)


@pytest.mark.parametrize("L", [1, 2, 4])
def test_unfused_design_long_terms_and_values_only(L):
    """The paper's three-kernel design on a system with terms of 10 factors
    (the cyclic10-shaped stand-in), with and without the Jacobian; refused
    before ph_eval_prepare sized its arrays, and on a second, larger call run
    in two chunks of the prepared capacity."""
    import torch
    s = synth.SHAPED["cyclic10"]()
    g = synth.gamma_of(s)
    S = ph.System(s)
    ph.eval_set_config(S, L, ph.EVAL_UNFUSED)
    with pytest.raises(ph.PHError, match="-1"):          # arrays not sized yet
        _eval(S, s, L, *synth.torus_points(s, 5, L, np.random.default_rng(1)), g)
    ph.eval_prepare(S, L, unfused_points=70)              # 128 points per chunk
    for npts in (70, 200):
        rng = np.random.default_rng(40 + npts)
        x, t = synth.torus_points(s, npts, L, rng)
        ov, oj, sv, sj = oracle.eval_homotopy(s, L, x, t, g)
        v, j = _eval(S, s, L, x, t, g)
        assert max(scaled_error(v, ov, sv), scaled_error(j, oj, sj)) <= TOL[L]
        val, none = ph.eval_jac(S, ph.to_soa(x), npts, L, torch.as_tensor(t, dtype=torch.float64).cuda(),
                                g, want_jac=False)
        torch.cuda.synchronize()
        assert none is None
        assert scaled_error(ph.from_soa(val, npts, (s.n_eq, 2, L)), ov, sv) <= TOL[L]


def test_inapplicable_kernel_is_refused():
    s = synth.eval_dense(seed=779, n=6, terms_per_eq=5, k=4)
    S = ph.System(s)
    rng = np.random.default_rng(12)
    x = synth.random_points(s.n_var, 70, 2, rng)
    ph.eval_set_config(S, 2, ph.EVAL_FAST_VECROW)     # double only
    with pytest.raises(ph.PHError, match="-4"):
        _eval(S, s, 2, x, rng.uniform(0, 1, 70), 1.0)
    x4 = synth.random_points(s.n_var, 70, 4, rng)
    ph.eval_set_config(S, 4, ph.EVAL_REGROW)          # double only
    with pytest.raises(ph.PHError, match="-4"):
        _eval(S, s, 4, x4, rng.uniform(0, 1, 70), 1.0)
    with pytest.raises(ph.PHError):
        ph.eval_set_config(S, 1, 7)


@pytest.mark.parametrize("L", [1, 2, 4])
def test_full_workload_every_launch_the_autotuner_may_pick(L):
    """The benchmark times the autotuner's choice on the full workload (n = 32,
    64 terms of 8 factors per equation, 65536 points): every (kernel, waves,
    groups) the autotuner can pick, at that size, against the oracle on a
    sample of points including both ends of the first tile and the last point."""
    import torch
    s = synth.eval_dense()
    npts = 65536
    x, t = synth.torus_points(s, npts, L)
    g = synth.gamma_of(s)
    S = ph.System(s)
    xs = ph.to_soa(x)
    tt = torch.as_tensor(t, dtype=torch.float64).cuda()
    nsamp = {1: 8, 2: 4, 4: 2}[L]
    idx = np.unique(np.concatenate([[0, 63, npts - 1],
                                    np.random.default_rng(21).integers(0, npts, nsamp)]))
    ov, oj, sv, sj = oracle.eval_homotopy(s, L, x[idx], t[idx], g)
    it = torch.as_tensor(idx, device="cuda")
    checked = 0
    for k in (ph.EVAL_FAST, ph.EVAL_FAST_VECROW, ph.EVAL_REGROW, ph.EVAL_GENERAL):
        for W in (1, 2, 4, 6, 8):
            for G in (1, 2, 4, 8):
                if W * G > s.n_eq:
                    continue
                ph.eval_set_config(S, L, k, W, G)
                try:
                    val, jm = ph.eval_jac(S, xs, npts, L, tt, g)
                except ph.PHError as e:
                    assert "-4" in str(e)            # the kernel does not apply here
                    continue
                torch.cuda.synchronize()
                v = val[:, it].T.contiguous().cpu().numpy().reshape(len(idx), s.n_eq, 2, L)
                j = jm[:, it].T.contiguous().cpu().numpy().reshape(len(idx), s.n_eq, s.n_var, 2, L)
                e = max(scaled_error(v, ov, sv), scaled_error(j, oj, sj))
                assert e <= TOL[L], (k, W, G, e)
                checked += 1
    ph.eval_set_config(S, L)
    assert checked >= 18 * {1: 3, 2: 2, 4: 2}[L]    # 18 tilings per applicable kernel
    print(f"[gpu] L={L} full workload, {checked} launch configurations match the oracle", flush=True)


def test_autotune_choice_persists_in_cache_file(tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("PH_AUTOTUNE_CACHE", str(cache))
    import torch
    s = synth.eval_dense(seed=780, n=8, terms_per_eq=20, k=4)
    L = 1
    rng = np.random.default_rng(13)
    npts = 4096
    x = synth.random_points(s.n_var, npts, L, rng, 0.95)
    t = rng.uniform(0, 1, npts)
    g = synth.gamma_of(s)
    S = ph.System(s)
    xs = ph.to_soa(x)
    tt = torch.as_tensor(t, dtype=torch.float64).cuda()
    ms = ph.eval_autotune(S, xs, npts, L, tt, g)
    assert ms > 0
    lines = cache.read_text().split("\n")
    fields = lines[0].split()
    assert fields[0] == "eval" and int(fields[3]) == L and int(fields[4]) in (1, 2, 3, 4)
    print(f"[gpu] autotune -> {lines[0]}", flush=True)
    # the tuned configuration still gives oracle-exact results
    idx = np.array([0, 1, 63, 64, 2000, npts - 1])
    v, j = _eval(S, s, L, x, t, g)
    ov, oj, sv, sj = oracle.eval_homotopy(s, L, x[idx], t[idx], g)
    assert max(scaled_error(v[idx], ov, sv), scaled_error(j[idx], oj, sj)) <= TOL[L]
    # a new handle of the same system finds the entry by fingerprint: pin the
    # general kernel with one wave through the file and check it is taken
    fields[4:7] = ["1", "1", "1"]
    cache.write_text(" ".join(fields) + "\n")
    S2 = ph.System(s)
    assert ph.eval_get_config(S2, L) == (1, 1, 1)      # read back from the file
    v2, j2 = _eval(S2, s, L, x, t, g)
    assert max(scaled_error(v2[idx], ov, sv), scaled_error(j2[idx], oj, sj)) <= TOL[L]
    # and an entry asking for a kernel that cannot run is honoured (and refused)
    s3 = synth.eval_dense(seed=781, n=6, terms_per_eq=5, k=4)
    S3 = ph.System(s3)
    x3 = synth.random_points(6, 64, 2, rng)
    t3 = rng.uniform(0, 1, 64)
    import torch as _t
    ph.eval_autotune(S3, ph.to_soa(x3), 64, 2, _t.as_tensor(t3, dtype=_t.float64).cuda(), g)
    last = cache.read_text().strip().split("\n")[-1].split()
    assert int(last[3]) == 2 and int(last[4]) in (1, 3)  # general kernel or DD fast path
    last[4] = "4"                                         # a double-only kernel
    cache.write_text(" ".join(last) + "\n")
    with pytest.raises(ph.PHError, match="-4"):
        _eval(ph.System(s3), s3, 2, x3, t3, g)


def test_track_autotune_choice_is_valid_and_cached(tmp_path, monkeypatch):
    """The tuned launch shape changes only the schedule: endpoints, status and
    step counts are bitwise those of the default shape; a second call reads
    the choice back from the cache file."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("PH_AUTOTUNE_CACHE", str(cache))
    small, cub = synth.tracking_small(), synth.tracking_cubic()
    systems = [ph.System(small), ph.System(cub)]
    gammas = [synth.gamma_of(small), synth.gamma_of(cub)]
    paths = [None, np.arange(0, 6561, 7)]
    base = ph.track_opts(prec=2, mixed=1)
    tuned, sec = ph.track_autotune(systems, gammas, paths, base, sample=400)
    assert sec > 0
    assert tuned.schedule in (ph.SCHED_PERSISTENT, ph.SCHED_GRAPH)
    assert 1 <= tuned.blocks_per_cu <= 16 and tuned.rounds_per_launch >= 1
    assert tuned.lanes_per_path in (0, 4, 8, 16, 32)
    assert (tuned.prec, tuned.mixed, tuned.h_max) == (2, 1, base.h_max)
    print(f"[gpu] tuned schedule={tuned.schedule} rounds={tuned.rounds_per_launch} "
          f"blocks_per_cu={tuned.blocks_per_cu} sample {sec:.3f} s", flush=True)
    a = ph.track_batch(systems, gammas, paths, base)
    b = ph.track_batch(systems, gammas, paths, tuned)
    assert (a["status"] == b["status"]).all() and (a["steps"] == b["steps"]).all()
    import torch
    assert torch.equal(a["x_end"], b["x_end"])
    again, sec2 = ph.track_autotune(systems, gammas, paths, base, sample=400)
    assert sec2 == 0.0
    assert (again.schedule, again.rounds_per_launch, again.blocks_per_cu, again.lanes_per_path) == \
        (tuned.schedule, tuned.rounds_per_launch, tuned.blocks_per_cu, tuned.lanes_per_path)
