"""Benchmark of the hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec 1|2|4]

A step is one ph_eval_jac launch over the evaluation workload: n = 32
equations and unknowns, 64 terms per equation over k = 8 distinct variables
with exponents 1..3, unit-modulus coefficients, 65536 points on the unit torus
with t ~ U[0,1) -- values and full Jacobian of gamma(1-t) g + t f.  Inputs are
resident in HBM before timing starts; the K launches are bracketed by HIP
events on the launch stream.  Prints ONE JSON line.

The roofline object uses algorithmic FP64 flops per point from the cost model
(per term: 3k-3+#{a>=2} complex products, k+1 complex additions, #{a>=2}+1
real scalings; flops per complex operation 6/2/2 in double, 80/40/16 in
double double, 660/212/124 in quad double as executed by the device
arithmetic) and compulsory bytes per point (x, t, H, J).  cpu_baseline is the
oracle (plain C, expansion arithmetic, symbolic derivatives) on a bounded
sample of the same points, on the host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6e12      # MI355X vector FP64 (FMA = 2 flops)
PEAK_HBM = 8.0e12        # bytes/s
CMUL = {1: 6, 2: 80, 4: 660}
CADD = {1: 2, 2: 40, 4: 212}
CSCALE = {1: 2, 2: 16, 4: 124}
PREC_NAME = {1: "complex double", 2: "complex double double", 4: "complex quad double"}


# HBM bytes per launch of the evaluation kernels from two rocprofv3 PMC runs
# (FETCH_SIZE, WRITE_SIZE), scaled by the factors a 2 GiB device copy gives
# (profiles/eval_*_n32_k8_65536pts.md).  Valid only for the kernel sources
# (the kernel's file and the headers it compiles) they were taken with: any
# change to them reports null.
TRAFFIC = {
    # the double kernel writes H and J once whatever its tiling
    "eval_d_pinned_kernel": {
        "bytes": 41433088 + 1107386368,   # read + write
        "sources": {"paper_1505_00383_amd/csrc/eval.hip": "a2fa63e42cb509a8",
                    "paper_1505_00383_amd/csrc/ph_arith.hpp": "1f4274c3666f77a9",
                    "paper_1505_00383_amd/csrc/ph_sweep.hpp": "afaab2dda7ee3e60",
                    "paper_1505_00383_amd/csrc/ph_internal.hpp": "ab9104fb80a39058"},
    },
    # the accumulation-register kernels stage x once per (point tile,
    # equation group): their reads depend on the tiling
    "eval_dd_arow_kernel": {
        "by_launch": {(3, 4, 1): 82423040 + 2214619008, (3, 4, 2): 147354795 + 2214631893,
                      (3, 4, 4): 281448320 + 2214658347},
        "sources": {"paper_1505_00383_amd/csrc/eval_dd.hip": "4f9b4854ab9300ef",
                    "paper_1505_00383_amd/csrc/ph_arow.hpp": "aee6853f608672f7",
                    "paper_1505_00383_amd/csrc/ph_arith.hpp": "1f4274c3666f77a9",
                    "paper_1505_00383_amd/csrc/ph_internal.hpp": "ab9104fb80a39058"},
    },
    "eval_qd_arow_kernel": {
        "by_launch": {(3, 4, 1): 170525531 + 4429184597, (3, 4, 2): 296279509 + 4429184597,
                      (3, 4, 4): 558127869 + 4429184597},
        "sources": {"paper_1505_00383_amd/csrc/eval_qd.hip": "fc3b726e4958d650",
                    "paper_1505_00383_amd/csrc/ph_arow.hpp": "aee6853f608672f7",
                    "paper_1505_00383_amd/csrc/ph_arith.hpp": "1f4274c3666f77a9",
                    "paper_1505_00383_amd/csrc/ph_internal.hpp": "ab9104fb80a39058"},
    },
}


def traffic_of(kernel, launch=None):
    import hashlib
    t = TRAFFIC.get(kernel)
    if t is None:
        return None
    if launch is not None and kernel in ("eval_dd_arow_kernel", "eval_qd_arow_kernel"):
        # these kernels run at most four waves per workgroup (one per SIMD):
        # a larger configured count launches four
        launch = (launch[0], min(launch[1], 4), launch[2])
    if "by_launch" in t and (launch is None or tuple(launch) not in t["by_launch"]):
        return None
    for path, sha in t["sources"].items():
        with open(os.path.join(ROOT, path), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest()[:16] != sha:
                return None
    return t["by_launch"][tuple(launch)] if "by_launch" in t else t["bytes"]


def flops_per_point(sysm, L):
    """Algorithmic FP64 flops of H and J at one point (cost model above),
    including the total-degree start terms x_i^{d_i} and -1."""
    fl = 0
    deg = sysm.degrees()
    terms = []
    for s in range(sysm.n_terms):
        a, b = sysm.term_fac_off[s], sysm.term_fac_off[s + 1]
        terms.append(list(sysm.fac_exp[a:b]))
    terms += [[int(d)] for d in deg] + [[] for _ in deg]
    for ex in terms:
        k = len(ex)
        n2 = sum(1 for e in ex if e >= 2)
        if k == 0:
            fl += CADD[L] + CSCALE[L]
            continue
        prods = 3 * k - 3 + n2
        fl += prods * CMUL[L] + (k + 1) * CADD[L] + (n2 + 1) * CSCALE[L]
    return fl


def bytes_per_point(sysm, L):
    n, m = sysm.n_var, sysm.n_eq
    return 16 * L * (n + m + m * n) + 8


def log(msg):
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_info():
    """Host cores the oracle may use and the CPU model (stated beside every
    oracle rate)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return {"nproc": avail, "cpu_count": os.cpu_count(), "model": model,
            "threads_used": min(16, avail)}


def mgs_flops(n, L):
    """FP64 flops of one least-squares Newton solve by MGS on the n x (n+1)
    augmented complex matrix [J | -H] in L limbs (the mixed scheme: L = 1),
    with its back substitution: n^2 (n+1) + n(n-1)/2 complex products and
    additions (projections, updates, back substitution), n^2 + n complex-by-
    real scalings (normalisation, division by r_kk), n^2 squared moduli."""
    cm = n * n * (n + 1) + n * (n - 1) // 2
    return cm * (CMUL[L] + CADD[L]) + (n * n + n) * CSCALE[L] + n * n * (CSCALE[L] + CADD[L] // 2)


def track_iteration_flops(sysm, L, mixed):
    """One evaluate-correct step of a path: H and J of the homotopy at one point
    in L limbs, the MGS solve (FP64 when mixed), the update of x in L limbs,
    and the FP64 norms of the convergence test."""
    n = sysm.n_var
    return flops_per_point(sysm, L) + mgs_flops(n, 1 if mixed else L) + n * CADD[L] + n * n + 4 * n


def predictor_flops(sysm, L, order):
    """One predictor step per path: the secant x + r (x - x_p) is one complex
    subtraction, scaling and addition per coordinate; order m >= 2 scales and
    adds m + 1 points."""
    n = sysm.n_var
    return n * (2 * CADD[L] + CSCALE[L]) if order <= 1 else n * (order + 1) * (CSCALE[L] + CADD[L])


def cpu_baseline(sysm, L, x, t, gamma, target_s=15.0):
    import oracle
    threads = min(16, os.cpu_count() or 1)
    # calibrate on one point, then size the sample for ~target_s of CPU work
    t0 = time.perf_counter()
    oracle.eval_homotopy(sysm, L, x[:1], t[:1], gamma, scales=False)
    one = time.perf_counter() - t0
    npts = int(max(threads, min(len(t), target_s / max(one, 1e-6))))
    npts = (npts // threads) * threads or threads
    t0 = time.perf_counter()
    oracle.eval_threaded(sysm, L, x[:npts], t[:npts], gamma, threads=threads)
    wall = time.perf_counter() - t0
    # one core, the paper's convention, on a smaller sample (about 3 s)
    m1 = int(max(1, min(len(t), 3.0 / max(one, 1e-6))))
    t0 = time.perf_counter()
    oracle.eval_homotopy(sysm, L, x[:m1], t[:m1], gamma, scales=False)
    one_rate = m1 / (time.perf_counter() - t0)
    hi = host_info()
    return {"value": npts / wall, "unit": "points/s", "cores": threads, "kind": "oracle",
            "sample": f"first {npts} of the 65536 points, {PREC_NAME[L]}, {threads} host threads "
                      f"over contiguous point ranges, {wall:.1f} s wall; one core: first {m1} points",
            "one_core_value": one_rate, "host": hi}


def time_eval(ph, torch, S, sysm, L, npts, steps, warmup, gamma, rng=None, inputs=None):
    from paper_1505_00383_amd import synth
    x, t = inputs if inputs is not None else synth.torus_points(sysm, npts, L, rng)
    xs = ph.to_soa(x)
    tt = torch.as_tensor(t, dtype=torch.float64).cuda()
    val = torch.empty((sysm.n_eq * 2 * L, npts), dtype=torch.float64, device="cuda")
    jac = torch.empty((sysm.n_eq * sysm.n_var * 2 * L, npts), dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        ph.eval_jac(S, xs, npts, L, tt, gamma, val=val, jac=jac)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(steps):
        ph.eval_jac(S, xs, npts, L, tt, gamma, val=val, jac=jac)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    ok = bool(torch.isfinite(val).all()) and bool(torch.isfinite(jac).all())
    return ms, ok, x, t


def track_roofline(sysm, L, mixed, order, rep, seconds, npaths):
    """Algorithmic FP64 flops per path from the device counters (Newton
    iterations and predictor steps, polish included) and the tracker's
    fraction of the FP64 vector peak."""
    it = track_iteration_flops(sysm, L, mixed)
    fl = rep["newton_its"] * it + rep["steps"] * predictor_flops(sysm, L, order)
    return {"flops_per_iteration": it, "flops_per_path": fl / max(npaths, 1),
            "achieved_TFLOPs": fl / seconds / 1e12, "fp64_frac": fl / seconds / PEAK_FP64}


def time_track(ph, torch, sysm, L, mixed, npaths, reps=1, order=1):
    """paths/s of ph_track on the first npaths start solutions (roots of unity),
    with the tracker's algorithmic flops and roofline fraction."""
    from paper_1505_00383_amd import synth
    S = ph.System(sysm)
    g = synth.gamma_of(sysm)
    opts = ph.track_opts(prec=L, mixed=mixed, predictor_order=order)
    ph.track(S, g, min(npaths, 64), opts)          # warm-up (module load, caches)
    st = torch.cuda.current_stream()
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        res = ph.track(S, g, npaths, opts)
        e1.record(st)
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) * 1e-3
        if best is None or sec < best[0]:
            best = (sec, res)
    sec, res = best
    rep = res["report"]
    return {"paths": npaths, "seconds": sec, "paths_per_s": npaths / sec,
            "success": int(rep["n_success"]), "failed_by_reason": {
                k: int(rep[k]) for k in ("n_diverged", "n_step_underflow", "n_max_steps",
                                         "n_singular", "n_nan")},
            "steps_per_path": rep["steps"] / max(npaths, 1),
            "steps_p50_p99_max": [float(np.percentile(res["steps"], 50)),
                                  float(np.percentile(res["steps"], 99)), int(res["steps"].max())],
            "newton_per_path": rep["newton_its"] / max(npaths, 1),
            "roofline": track_roofline(sysm, L, mixed, order, rep, sec, npaths)}, res


def longest_path_alone(ph, torch, sysm, L, mixed, res, whole_s, reps=2):
    """The path with the most steps in ``res``, tracked by itself from its own
    start point: when this takes nearly as long as the whole run, paths/s on
    that workload is set by one path's step latency, not by throughput."""
    from paper_1505_00383_amd import synth
    S = ph.System(sysm)
    g = synth.gamma_of(sysm)
    opts = ph.track_opts(prec=L, mixed=mixed)
    i = int(np.argmax(res["steps"]))
    xs = ph.start_solutions(S, L, i, 1)
    st = torch.cuda.current_stream()
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        r1 = ph.track(S, g, 1, opts, x_start=xs)
        e1.record(st)
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) * 1e-3
        best = sec if best is None else min(best, sec)
    return {"path": i, "steps": int(r1["steps"][0]), "seconds": best,
            "fraction_of_whole_run": best / whole_s}


def _limb_err(xg, xr):
    """||xg - xr||_inf / max(1, ||xr||_inf) per path for [p, n, 2, L] limb arrays,
    each limb difference summed exactly (math.fsum) before rounding."""
    import math
    p, n = xg.shape[0], xg.shape[1]
    out = np.zeros(p)
    for k in range(p):
        worst, big = 0.0, 1.0
        for i in range(n):
            dre = math.fsum(list(xg[k, i, 0]) + [-v for v in xr[k, i, 0]])
            dim = math.fsum(list(xg[k, i, 1]) + [-v for v in xr[k, i, 1]])
            worst = max(worst, math.hypot(dre, dim))
            big = max(big, math.hypot(xr[k, i, 0].sum(), xr[k, i, 1].sum()))
        out[k] = worst / big
    return out


def oracle_track_rate(sysm, gamma, L, mixed, paths, threads):
    """The oracle's tracker (plain C, expansion arithmetic) on the listed start
    paths with `threads` host threads; returns (paths/s, result)."""
    import oracle
    t0 = time.perf_counter()
    r = oracle.track(sysm, gamma, np.asarray(paths), oracle.Opts(prec=L, mixed=mixed), threads=threads)
    return len(paths) / (time.perf_counter() - t0), r


def oracle_beside(sysm, gamma, L, mixed, one_paths, all_paths, gpu_res=None, gpu_paths=None):
    """One-core and all-core oracle tracking rates on stated path subsets, and,
    for a mixed GPU run, the error of every GPU endpoint of the all-core
    subset against the oracle's PLAIN track in the same precision."""
    import paper_1505_00383_amd as ph
    hi = host_info()
    thr = hi["threads_used"]
    r1, _ = oracle_track_rate(sysm, gamma, L, mixed, one_paths, 1)
    ref_mixed = mixed if gpu_res is None else 0            # endpoint errors: plain reference
    ra, ref = oracle_track_rate(sysm, gamma, L, ref_mixed, all_paths, thr)
    out = {"oracle_1core_paths_per_s": r1, "oracle_1core_sample": f"paths {list(map(int, one_paths))}",
           "oracle_1core_mixed": int(mixed),
           "oracle_allcores_paths_per_s": ra, "oracle_allcores_threads": thr,
           "oracle_allcores_sample": f"{len(all_paths)} paths (every {max(1, int(all_paths[1] - all_paths[0])) if len(all_paths) > 1 else 1}th from {int(all_paths[0])})",
           "oracle_allcores_mixed": int(ref_mixed)}
    if gpu_res is not None:
        import torch
        pos = np.searchsorted(gpu_paths, all_paths)
        it = torch.as_tensor(pos, device="cuda")
        xg = ph.from_soa(gpu_res["x_end"][:, it], len(pos), (sysm.n_var, 2, L))
        st = gpu_res["status"][pos]
        ok = (st == 1) & (ref["status"] == 1)
        err = _limb_err(xg[ok], ref["x"][ok]) if ok.any() else np.zeros(0)
        out["mixed_endpoint_error_vs_oracle_plain"] = {
            "paths": int(len(pos)), "both_succeeded": int(ok.sum()),
            "status_agree": int(np.sum(st == ref["status"])),
            "max": float(err.max()) if err.size else None,
            "median": float(np.median(err)) if err.size else None}
    return out


def endpoint_agreement(ph, a, b, n, L, npaths, tol):
    xa = ph.from_soa(a["x_end"], npaths, (n, 2, L)).sum(-1)
    xb = ph.from_soa(b["x_end"], npaths, (n, 2, L)).sum(-1)
    ok = (a["status"] == 1) & (b["status"] == 1)
    d = np.abs(xa - xb).max(-1).max(-1) / np.maximum(1.0, np.abs(xb).max(-1).max(-1))
    return float(np.mean(ok & (d <= tol)))


def batch_roofline(sysms, res, order, seconds, L=2, mixed=1):
    """Algorithmic flops of a batch: every path's predictor steps (device
    array) times its system's cost per step, the Newton iterations spread over
    the steps at the batch's measured ratio (the device counts them in total)."""
    rep = res["report"]
    off = res["path_off"]
    steps = res["steps"].astype(np.float64)
    ratio = rep["newton_its"] / max(rep["steps"], 1)
    fl = 0.0
    for k, sy in enumerate(sysms):
        st_k = steps[off[k]:off[k + 1]].sum()
        fl += st_k * (ratio * track_iteration_flops(sy, L, mixed) + predictor_flops(sy, L, order))
    total = int(off[-1])
    return {"flops_per_path": fl / max(total, 1), "achieved_TFLOPs": fl / seconds / 1e12,
            "fp64_frac": fl / seconds / PEAK_FP64}


def time_batch(ph, torch, systems, gammas, paths, opts, sysms=None):
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    res = ph.track_batch(systems, gammas, paths, opts)
    e1.record(st)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3
    rep = res["report"]
    total = int(res["path_off"][-1])
    out = {"paths": total, "seconds": sec, "paths_per_s": total / sec,
           "success": int(rep["n_success"]), "failed_by_reason": {
               k: int(rep[k]) for k in ("n_diverged", "n_step_underflow", "n_max_steps",
                                        "n_singular", "n_nan")},
           "steps_per_path": rep["steps"] / max(total, 1),
           "newton_per_path": rep["newton_its"] / max(total, 1)}
    if sysms is not None:
        out["roofline"] = batch_roofline(sysms, res, opts.predictor_order, sec, opts.prec, opts.mixed)
    return out, res


def batch_oracle(sysms, gammas, paths, res):
    """The oracle on (system, path) pairs sampled across the batch: one core in
    the GPU run's mode (DD residual, FP64 solves), all host cores in plain DD,
    whose endpoints are the reference for the GPU's mixed endpoints."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    import paper_1505_00383_amd as ph
    import torch
    hi = host_info()
    thr = hi["threads_used"]
    rng = np.random.default_rng(99)
    pairs = [(int(k), int(rng.integers(0, len(paths[k])))) for k in rng.choice(len(sysms), 2 * thr)]

    def one(pr, mixed):
        k, j = pr
        return oracle.track(sysms[k], gammas[k], paths[k][j:j + 1], oracle.Opts(prec=2, mixed=mixed))

    t0 = time.perf_counter()
    for pr in pairs[:4]:
        one(pr, 1)
    r1 = 4 / (time.perf_counter() - t0)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(thr) as ex:
        refs = list(ex.map(lambda pr: one(pr, 0), pairs))
    ra = len(pairs) / (time.perf_counter() - t0)
    off = res["path_off"]
    errs, agree = [], 0
    for (k, j), ref in zip(pairs, refs):
        gi = int(off[k]) + j
        n = sysms[k].n_var
        xg = ph.from_soa(res["x_end"][:n * 2 * 2, gi:gi + 1], 1, (n, 2, 2))
        agree += int(res["status"][gi] == ref["status"][0])
        if res["status"][gi] == 1 and ref["status"][0] == 1:
            errs.append(_limb_err(xg, ref["x"])[0])
    errs = np.array(errs)
    return {"oracle_1core_paths_per_s": r1, "oracle_1core_sample": "4 sampled (system, path) pairs, DD mixed",
            "oracle_allcores_paths_per_s": ra, "oracle_allcores_threads": thr,
            "oracle_allcores_sample": f"{len(pairs)} sampled (system, path) pairs, plain DD",
            "mixed_endpoint_error_vs_oracle_plain": {
                "paths": len(pairs), "both_succeeded": int(errs.size), "status_agree": agree,
                "max": float(errs.max()) if errs.size else None,
                "median": float(np.median(errs)) if errs.size else None}}


def batch_extra(ph, torch, cpu=True):
    """64 systems, n ~ U{4..16}, d ~ U{2,3}, 8..32 terms per equation, about
    200k paths in one launch, DD residual with FP64 Newton solves; the launch
    shape is autotuned on a 16384-path sample, then the whole batch runs
    under the graph schedule and the persistent schedule."""
    from paper_1505_00383_amd import synth
    sysms, gammas, paths, cap = synth.batch_heterogeneous()
    systems = [ph.System(s) for s in sysms]
    base = ph.track_opts(prec=2, mixed=1)
    tuned, tsec = ph.track_autotune(systems, gammas, paths, base, sample=16384)
    # graph schedule: launches ended by the default time budget, and by a
    # fixed round count (every wave waits for the slowest at each boundary)
    graph = ph.track_opts(prec=2, mixed=1, schedule=ph.SCHED_GRAPH,
                          blocks_per_cu=tuned.blocks_per_cu)
    graph_fixed = ph.track_opts(prec=2, mixed=1, schedule=ph.SCHED_GRAPH,
                                blocks_per_cu=tuned.blocks_per_cu, rounds_per_launch=32,
                                launch_ms=0.0)
    out = {"systems": len(sysms), "cap": int(cap),
           "n_hist": {int(n): int(sum(1 for s in sysms if s.n_var == n))
                      for n in sorted({s.n_var for s in sysms})},
           "tuned": {"schedule": "graph" if tuned.schedule == ph.SCHED_GRAPH else "persistent",
                     "rounds_per_launch": tuned.rounds_per_launch, "launch_ms": tuned.launch_ms,
                     "blocks_per_cu": tuned.blocks_per_cu, "sample_seconds": tsec}}
    out["tuned_run"], res = time_batch(ph, torch, systems, gammas, paths, tuned, sysms)
    out["graph"], _ = time_batch(ph, torch, systems, gammas, paths, graph, sysms)
    out["graph_32_rounds_per_launch"], _ = time_batch(ph, torch, systems, gammas, paths, graph_fixed, sysms)
    out["persistent_default"], _ = time_batch(ph, torch, systems, gammas, paths, base, sysms)
    if cpu:
        out["oracle"] = batch_oracle(sysms, gammas, paths, res)
    return out


def hbm_extra(ph, torch, steps):
    """Double-precision eval of the n = 16, degree-2 tracking system (k <= 2)
    at 2^20 points: about 1 flop per compulsory byte, so HBM-bound."""
    from paper_1505_00383_amd import synth
    s = synth.tracking_quadratic16()
    npts = 1 << 20
    S = ph.System(s)
    rng = np.random.Generator(np.random.PCG64(synth.SEED_BASE + 3))
    ms, ok, _, _ = time_eval(ph, torch, S, s, 1, npts, steps, 2, synth.gamma_of(s), rng)
    bpp = bytes_per_point(s, 1)
    fpp = flops_per_point(s, 1)
    return {"points": npts, "ms": ms, "points_per_s": npts / (ms * 1e-3),
            "bytes_per_point": bpp, "flops_per_point": fpp,
            "hbm_GBps_compulsory": bpp * npts / (ms * 1e-3) / 1e9,
            "hbm_frac_compulsory": bpp * npts / (ms * 1e-3) / PEAK_HBM, "finite": ok}


def pcie_extra(ph, torch, S, sysm, L, npts, gamma, reps=5):
    """The rate a caller holding its points in host memory sees: copy x and t
    from pinned host buffers, evaluate, copy H and J back, all on one stream.
    Not the benchmark value (that one starts with the inputs in HBM)."""
    from paper_1505_00383_amd import synth
    x, t = synth.torus_points(sysm, npts, L)
    xs_host = ph.to_soa(x, device="cpu").pin_memory()
    t_host = torch.as_tensor(t, dtype=torch.float64).pin_memory()
    xs = torch.empty_like(xs_host, device="cuda")
    tt = torch.empty_like(t_host, device="cuda")
    val = torch.empty((sysm.n_eq * 2 * L, npts), dtype=torch.float64, device="cuda")
    jac = torch.empty((sysm.n_eq * sysm.n_var * 2 * L, npts), dtype=torch.float64, device="cuda")
    val_host = torch.empty(val.shape, dtype=torch.float64, pin_memory=True)
    jac_host = torch.empty(jac.shape, dtype=torch.float64, pin_memory=True)

    def one():
        xs.copy_(xs_host, non_blocking=True)
        tt.copy_(t_host, non_blocking=True)
        ph.eval_jac(S, xs, npts, L, tt, gamma, val=val, jac=jac)
        val_host.copy_(val, non_blocking=True)
        jac_host.copy_(jac, non_blocking=True)

    one()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        one()
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    moved = xs_host.numel() * 8 + t_host.numel() * 8 + val.numel() * 8 + jac.numel() * 8
    return {"points": npts, "ms": ms, "points_per_s": npts / (ms * 1e-3),
            "bytes_over_pcie": moved, "GBps_over_pcie_incl_eval": moved / (ms * 1e-3) / 1e9,
            "finite": bool(torch.isfinite(jac_host).all())}


# The paper's own speedups of its GPU evaluation over one CPU core (Tables
# of Section 4, a Tesla K20C against one core of a Xeon E5-2670): context for
# the stand-ins of the same shape, not a target.
PAPER_EVAL_SPEEDUP = {"cyclic10": {1: 13.50, 2: 77.47, 4: 99.44},
                      "nash8": {1: 13.97, 2: 81.75, 4: 95.07},
                      "pieri44": {1: 14.67, 2: 81.60, 4: 89.79}}


def unfused_extra(ph, torch, S, sysm, gamma, steps):
    """The paper's three-kernel design (coeff / mon / sum with the products
    stored in device memory) against the fused kernel on the benchmark
    workload, D and DD; the bytes its intermediate arrays move per point."""
    out = {}
    npts = 65536
    slots = sum(int(sysm.term_fac_off[s + 1] - sysm.term_fac_off[s]) + 1 for s in range(sysm.n_terms))
    slots += 3 * sysm.n_eq                   # start terms x_i^d (2 slots) and -1 (1 slot)
    terms = sysm.n_terms + 2 * sysm.n_eq
    for L in (1, 2):
        ph.eval_set_config(S, L, ph.EVAL_UNFUSED)
        ph.eval_prepare(S, L, unfused_points=npts)
        ms, ok, _, _ = time_eval(ph, torch, S, sysm, L, npts, steps, 1, gamma)
        ph.eval_set_config(S, L)
        fused, _, _, _ = time_eval(ph, torch, S, sysm, L, npts, steps, 1, gamma)
        inter = 16 * L * (2 * terms + 2 * slots)   # cff written + read, slots written + read
        out[PREC_NAME[L]] = {"unfused_ms": ms, "fused_ms": fused, "fusion_speedup": ms / fused,
                             "intermediate_bytes_per_point": inter,
                             "unfused_intermediate_GBps": inter * npts / (ms * 1e-3) / 1e9,
                             "finite": ok}
    return out


def paper_shaped_extra(ph, torch, cpu_seconds=1.0):
    """Evaluation of the stand-ins shaped like the paper's benchmark systems at
    as many points as the paper has paths, in D/DD/QD, beside the oracle on
    ONE host core (the paper's convention) on a bounded sample."""
    import oracle
    from paper_1505_00383_amd import synth
    out = {}
    for name, make in synth.SHAPED.items():
        s = make()
        g = synth.gamma_of(s)
        S = ph.System(s)
        npts = int(s.meta["paths"])
        row = {"n": s.n_var, "monomials": s.n_terms, "points": npts}
        for L in (1, 2, 4):
            rng = np.random.Generator(np.random.PCG64(synth.SEED_BASE + 20 + L))
            ms, ok, x, t = time_eval(ph, torch, S, s, L, npts, 5, 1, g, rng)
            t0 = time.perf_counter()
            oracle.eval_homotopy(s, L, x[:1], t[:1], g, scales=False)
            one = time.perf_counter() - t0
            m = max(1, min(64, int(cpu_seconds / max(one, 1e-6))))
            t0 = time.perf_counter()
            oracle.eval_homotopy(s, L, x[:m], t[:m], g, scales=False)
            cpu = m / (time.perf_counter() - t0)
            gpu = npts / (ms * 1e-3)
            row[PREC_NAME[L]] = {"gpu_points_per_s": gpu, "ms": ms, "finite": ok,
                                 "oracle_1core_points_per_s": cpu, "oracle_sample_points": m,
                                 "speedup_vs_1core_oracle": gpu / cpu,
                                 "paper_speedup_k20c_vs_1core_context": PAPER_EVAL_SPEEDUP[name][L]}
        out[name] = row
    return out


def tracking_extras(ph, torch, cpu=True):
    """Tracking on the four tracking workloads: paths/s, algorithmic flops per
    path and roofline fraction (device counters), mixed vs plain, and the
    oracle timed beside it on stated path subsets (one core and all host
    cores), with the error of every mixed endpoint of the subset against the
    oracle's plain track in the same precision."""
    from paper_1505_00383_amd import synth
    out = {}
    thr = host_info()["threads_used"]
    small = synth.tracking_small()
    d_small, _ = time_track(ph, torch, small, 1, 0, 8, reps=3)
    if cpu:
        d_small["oracle"] = oracle_beside(small, synth.gamma_of(small), 1, 0, np.arange(8), np.arange(8))
    out["track_n3_d2_8paths_double"] = d_small
    log("tracking n = 3 done")
    cub = synth.tracking_cubic()
    gc = synth.gamma_of(cub)
    B = 3 ** 8
    dd_m, r_m = time_track(ph, torch, cub, 2, 1, B, reps=2)
    dd_p, r_p = time_track(ph, torch, cub, 2, 0, B, reps=2)
    d_p, r_d = time_track(ph, torch, cub, 1, 0, B, reps=2)
    d_p["longest_path_alone"] = longest_path_alone(ph, torch, cub, 1, 0, r_d, d_p["seconds"])
    dd_m["longest_path_alone"] = longest_path_alone(ph, torch, cub, 2, 1, r_m, dd_m["seconds"])
    row = {"double_plain": d_p, "dd_mixed": dd_m, "dd_plain": dd_p,
           "dd_mixed_over_plain": dd_m["paths_per_s"] / dd_p["paths_per_s"],
           "dd_endpoint_agreement_1e-24": endpoint_agreement(ph, r_m, r_p, 8, 2, B, 1e-24)}
    if cpu:
        sub = np.arange(4 * thr) * (B // (4 * thr))
        row["oracle"] = oracle_beside(cub, gc, 2, 1, np.arange(6), sub, r_m, np.arange(B))
    out["track_n8_d3_6561paths"] = row
    log("tracking n = 8 done")
    q16 = synth.tracking_quadratic16()
    gq = synth.gamma_of(q16)
    sub = 4096
    qd_m, q_m = time_track(ph, torch, q16, 4, 1, sub)
    qd_p, q_p = time_track(ph, torch, q16, 4, 0, sub)
    out["track_n16_d2_qd_4096paths"] = {
        "qd_mixed": qd_m, "qd_plain": qd_p,
        "qd_mixed_over_plain": qd_m["paths_per_s"] / qd_p["paths_per_s"],
        "qd_endpoint_agreement_1e-48": endpoint_agreement(ph, q_m, q_p, 16, 4, sub, 1e-48)}
    full, r_full = time_track(ph, torch, q16, 4, 1, 2 ** 16)
    if cpu:
        sub16 = np.arange(thr) * (2 ** 16 // thr)
        full["oracle"] = oracle_beside(q16, gq, 4, 1, np.arange(2), sub16, r_full, np.arange(2 ** 16))
    out["track_n16_d2_qd_mixed_65536paths"] = full
    log("tracking n = 16 done")
    # the fourth-order predictor (current and four previous points)
    c4, _ = time_track(ph, torch, cub, 2, 1, B, reps=2, order=4)
    f4, _ = time_track(ph, torch, q16, 4, 1, 2 ** 16, order=4)
    out["predictor_order4"] = {
        "track_n8_d3_6561paths_dd_mixed": c4,
        "over_secant_n8_d3": c4["paths_per_s"] / dd_m["paths_per_s"],
        "track_n16_d2_65536paths_qd_mixed": f4,
        "over_secant_n16_d2": f4["paths_per_s"] / full["paths_per_s"]}
    return out


def profile_mode(ph, torch, mode):
    """One run of a single workload, printing what it did (for rocprofv3)."""
    from paper_1505_00383_amd import synth
    if mode == "copy":
        n = (2 << 30) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        st = torch.cuda.current_stream()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        b.copy_(a)                      # first copy: page-in, not timed
        ev[0].record(st)
        for _ in range(2):
            b.copy_(a)
        ev[1].record(st)
        # the practical write-only rate (the evaluation kernels mostly write)
        ev[2].record(st)
        for _ in range(2):
            b.fill_(0.5)
        ev[3].record(st)
        torch.cuda.synchronize()
        copy_s = ev[0].elapsed_time(ev[1]) * 1e-3 / 2
        fill_s = ev[2].elapsed_time(ev[3]) * 1e-3 / 2
        print(json.dumps({"mode": mode, "bytes_read_per_copy": n * 8, "bytes_written_per_copy": n * 8,
                          "copies": 3, "copy_GBps_read_plus_write": 2 * n * 8 / copy_s / 1e9,
                          "fill_GBps_write": n * 8 / fill_s / 1e9}))
        return
    if mode == "eval_hbm":
        print(json.dumps({"mode": mode, **hbm_extra(ph, torch, 20)}))
        return
    if mode == "track_n8_dd":
        s = synth.tracking_cubic()
        res = ph.track(ph.System(s), synth.gamma_of(s), 6561, ph.track_opts(prec=2, mixed=1))
        print(json.dumps({"mode": mode, "report": res["report"]}))
        return
    if mode == "track_n8_dd_longest":
        # the whole workload once (its last dispatch is not the one to read),
        # then the path with the most steps by itself: the last track_kernel
        # dispatch of this mode
        s = synth.tracking_cubic()
        S, g = ph.System(s), synth.gamma_of(s)
        opts = ph.track_opts(prec=2, mixed=1)
        res = ph.track(S, g, 6561, opts)
        i = int(np.argmax(res["steps"]))
        one = ph.track(S, g, 1, opts, x_start=ph.start_solutions(S, 2, i, 1))
        print(json.dumps({"mode": mode, "path": i, "report": one["report"]}))
        return
    if mode == "track_n16_qd":
        s = synth.tracking_quadratic16()
        res = ph.track(ph.System(s), synth.gamma_of(s), 2 ** 16, ph.track_opts(prec=4, mixed=1))
        print(json.dumps({"mode": mode, "report": res["report"]}))
        return
    sysms, gammas, paths, cap = synth.batch_heterogeneous()
    systems = [ph.System(x) for x in sysms]
    res = ph.track_batch(systems, gammas, paths,
                         ph.track_opts(prec=2, mixed=1, schedule=ph.SCHED_GRAPH))
    print(json.dumps({"mode": mode, "report": res["report"]}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--prec", type=int, default=1, choices=[1, 2, 4])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the library's default kernel choice instead of the autotuned one")
    ap.add_argument("--kernel", type=int, default=0,
                    help="evaluation kernel choice of ph_eval_set_config for the timed launches "
                         "(0 automatic; 5 the unfused three-kernel design)")
    ap.add_argument("--waves", type=int, default=0,
                    help="with --kernel: waves per workgroup (0: the library's default)")
    ap.add_argument("--groups", type=int, default=0,
                    help="with --kernel: equation groups (0: the library's default)")
    ap.add_argument("--mode", default="eval",
                    choices=["eval", "eval_hbm", "track_n8_dd", "track_n8_dd_longest", "track_n16_qd", "track_batch", "copy"],
                    help="eval: the benchmark line; the others run one workload for profiling: "
                         "the HBM-bound n = 16 evaluation at 2^20 points, the 6561-path DD-mixed "
                         "tracking of the n = 8 cubic system (or its longest path by itself), "
                         "the 65536-path QD-mixed "
                         "tracking, the 64-system batch, or a device copy of 2 GiB (calibrates "
                         "the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): paths and "
              f"points shard across GPUs with no exchange until a final gather, which is a "
              f"design here, not an implemented launcher.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1505_00383_amd as ph
    from paper_1505_00383_amd import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.mode != "eval":
        profile_mode(ph, torch, args.mode)
        return
    L = args.prec
    sysm = synth.eval_dense()
    gamma = synth.gamma_of(sysm)
    npts = 65536
    S = ph.System(sysm)
    tuned_cfg = None
    # inputs first: the GPU goes from tuning straight into the warm-up and the
    # timed launches, with no idle gap (its clock drops when it idles)
    x0, t0 = synth.torus_points(sysm, npts, L)
    if args.kernel:
        ph.eval_set_config(S, L, args.kernel, args.waves, args.groups)
        if args.kernel == ph.EVAL_UNFUSED:
            ph.eval_prepare(S, L, unfused_points=npts)
    elif not args.no_autotune:
        # the library's autotuner picks kernel and tiling on this workload; a
        # choice already in the PH_AUTOTUNE_CACHE file is taken as it is
        tuned_cfg = ph.eval_get_config(S, L)
        tuned_by = "ph_eval_autotune (cache file)"
        if tuned_cfg[0] == 0:
            ph.eval_autotune(S, ph.to_soa(x0), npts, L, torch.as_tensor(t0, dtype=torch.float64).cuda(), gamma)
            tuned_cfg = ph.eval_get_config(S, L)
            tuned_by = "ph_eval_autotune"
    ms, ok, x, t = time_eval(ph, torch, S, sysm, L, npts, args.steps, args.warmup, gamma, inputs=(x0, t0))
    log(f"timed eval prec {L}: {ms:.4f} ms per step")
    if args.kernel:
        ph.eval_set_config(S, L)
    fpp = flops_per_point(sysm, L)
    bpp = bytes_per_point(sysm, L)
    secs = ms * 1e-3
    achieved = fpp * npts / secs
    fast = {1: "eval_d_pinned_kernel", 2: "eval_dd_arow_kernel", 4: "eval_qd_arow_kernel"}
    kname = fast.get(L, f"eval_kernel<{L},8,true,true>")
    kchoice = args.kernel or (tuned_cfg[0] if tuned_cfg else 0)
    if kchoice:
        kname = {1: f"eval_kernel<{L},8,true,true>", 2: "eval_d_regrow_kernel<8>", 3: fast.get(L),
                 4: "eval_d_fast_kernel", 5: "coeff_kernel + mon_kernel + sum_kernel"}[kchoice]
    traffic = traffic_of(kname, tuned_cfg)
    result = {
        "metric": "eval+Jacobian points/sec (paths/sec to t=1 in extras), per precision",
        "value": npts / secs,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"eval+jacobian of gamma(1-t)g+t f, n=32, 64 terms/eq over k=8 "
                               f"vars, exponents 1..3, 65536 torus points, {PREC_NAME[L]}",
                   "prec_limbs": L, "points": npts, "n": 32, "terms": int(sysm.n_terms),
                   "parallelism": "single GPU"},
        "launch": ({"kernel": tuned_cfg[0], "waves_per_workgroup": tuned_cfg[1],
                    "equation_groups": tuned_cfg[2], "chosen_by": tuned_by}
                   if tuned_cfg else {"chosen_by": "--kernel" if args.kernel else "default"}),
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64, "traffic": traffic,
                     "traffic_unit": "bytes per launch", "kernel": kname,
                     "flops_per_point": fpp, "bytes_per_point": bpp,
                     "hbm_GBps_compulsory": bpp * npts / secs / 1e9,
                     "hbm_frac_compulsory": bpp * npts / secs / PEAK_HBM},
        "finite": ok,
    }
    if not args.no_extras:
        extras = {}
        for L2 in (1, 2, 4):
            if L2 == L:
                continue
            cfg2 = None
            x2, t2 = synth.torus_points(sysm, npts, L2)
            if not args.no_autotune:
                cfg2 = ph.eval_get_config(S, L2)
                if cfg2[0] == 0:
                    ph.eval_autotune(S, ph.to_soa(x2), npts, L2,
                                     torch.as_tensor(t2, dtype=torch.float64).cuda(), gamma)
                    cfg2 = ph.eval_get_config(S, L2)
            ms2, ok2, _, _ = time_eval(ph, torch, S, sysm, L2, npts, max(3, args.steps // 4), 3, gamma,
                                       inputs=(x2, t2))
            f2 = flops_per_point(sysm, L2)
            log(f"eval prec {L2}: {ms2:.3f} ms")
            k2 = {1: f"eval_kernel<{L2},8,true,true>", 2: "eval_d_regrow_kernel<8>",
                  3: {1: "eval_d_pinned_kernel", 2: "eval_dd_arow_kernel",
                      4: "eval_qd_arow_kernel"}[L2]}.get(cfg2[0] if cfg2 else 3)
            t2 = traffic_of(k2, cfg2)
            extras[f"eval_prec{L2}"] = {"points_per_s": npts / (ms2 * 1e-3), "ms": ms2,
                                        "fp64_frac": f2 * npts / (ms2 * 1e-3) / PEAK_FP64,
                                        "launch": cfg2, "kernel": k2, "traffic": t2,
                                        "traffic_over_compulsory":
                                            t2 / (bytes_per_point(sysm, L2) * npts) if t2 else None,
                                        "finite": ok2}
        extras["eval_n16_d2_hbm_1M_points_double"] = hbm_extra(ph, torch, max(3, args.steps // 4))
        log("hbm-bound eval done")
        extras["eval_pcie_inclusive_host_buffers"] = pcie_extra(ph, torch, S, sysm, L, npts, gamma)
        extras["unfused_three_kernel_ablation"] = unfused_extra(ph, torch, S, sysm, gamma, 5)
        log("unfused ablation done")
        extras.update(tracking_extras(ph, torch, cpu=not args.no_cpu_baseline))
        log("tracking workloads done")
        extras["track_batch64_dd_mixed"] = batch_extra(ph, torch, cpu=not args.no_cpu_baseline)
        log("batch done")
        if not args.no_cpu_baseline:
            extras["paper_shaped_eval"] = paper_shaped_extra(ph, torch)
        result["extras"] = extras
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(sysm, L, x, t, gamma)
    # the compact per-precision summary comes last, so a truncated log keeps it
    result["summary"] = summary(result, L)
    print(json.dumps(result))


def summary(result, L):
    """Every cell of the metric in one place: evaluation points/s and FP64
    fraction per precision, tracking paths/s and FP64 fraction per workload
    (mixed and plain), the oracle's tracking rates beside them, and the
    error of the mixed endpoints against the oracle's plain track."""
    name = {1: "D", 2: "DD", 4: "QD"}
    ex = result.get("extras", {})
    rl = result["roofline"]
    out = {"eval_points_per_s": {name[L]: result["value"]},
           "eval_fp64_frac": {name[L]: rl["frac"]},
           "eval_traffic_over_compulsory": {
               name[L]: rl["traffic"] / (rl["bytes_per_point"] * result["config"]["points"])
               if rl.get("traffic") else None}}
    for L2 in (1, 2, 4):
        e = ex.get(f"eval_prec{L2}")
        if e:
            out["eval_points_per_s"][name[L2]] = e["points_per_s"]
            out["eval_fp64_frac"][name[L2]] = e["fp64_frac"]
            out["eval_traffic_over_compulsory"][name[L2]] = e.get("traffic_over_compulsory")
    runs = {}
    if "track_n3_d2_8paths_double" in ex:
        runs["n3_d2_8p_D_plain"] = ex["track_n3_d2_8paths_double"]
    c = ex.get("track_n8_d3_6561paths", {})
    for k, lab in (("double_plain", "n8_d3_6561p_D_plain"), ("dd_mixed", "n8_d3_6561p_DD_mixed"),
                   ("dd_plain", "n8_d3_6561p_DD_plain")):
        if k in c:
            runs[lab] = c[k]
    q = ex.get("track_n16_d2_qd_4096paths", {})
    for k, lab in (("qd_mixed", "n16_d2_4096p_QD_mixed"), ("qd_plain", "n16_d2_4096p_QD_plain")):
        if k in q:
            runs[lab] = q[k]
    if "track_n16_d2_qd_mixed_65536paths" in ex:
        runs["n16_d2_65536p_QD_mixed"] = ex["track_n16_d2_qd_mixed_65536paths"]
    b = ex.get("track_batch64_dd_mixed", {})
    if "tuned_run" in b:
        runs["batch64_200kp_DD_mixed"] = b["tuned_run"]
    if runs:
        out["track_paths_per_s"] = {k: v["paths_per_s"] for k, v in runs.items()}
        out["track_fp64_frac"] = {k: v["roofline"]["fp64_frac"] for k, v in runs.items() if "roofline" in v}
        out["track_longest_path_alone_over_whole_run"] = {
            k: v["longest_path_alone"]["fraction_of_whole_run"] for k, v in runs.items()
            if "longest_path_alone" in v}
    orc = {"n3_d2_D": ex.get("track_n3_d2_8paths_double", {}).get("oracle"),
           "n8_d3_DD": c.get("oracle"),
           "n16_d2_QD": ex.get("track_n16_d2_qd_mixed_65536paths", {}).get("oracle"),
           "batch64_DD": b.get("oracle")}
    orc = {k: v for k, v in orc.items() if v}
    if orc:
        out["oracle_track_paths_per_s"] = {
            k: {"1core": v["oracle_1core_paths_per_s"], "allcores": v["oracle_allcores_paths_per_s"],
                "threads": v["oracle_allcores_threads"]} for k, v in orc.items()}
        out["mixed_endpoint_err_vs_oracle_plain"] = {
            k: {"max": v["mixed_endpoint_error_vs_oracle_plain"]["max"],
                "median": v["mixed_endpoint_error_vs_oracle_plain"]["median"],
                "paths": v["mixed_endpoint_error_vs_oracle_plain"]["paths"]}
            for k, v in orc.items() if "mixed_endpoint_error_vs_oracle_plain" in v}
    if "cpu_baseline" in result:
        out["oracle_eval_points_per_s"] = {"allcores": result["cpu_baseline"]["value"],
                                           "1core": result["cpu_baseline"]["one_core_value"]}
        out["host"] = result["cpu_baseline"].get("host")
    return out


if __name__ == "__main__":
    main()
