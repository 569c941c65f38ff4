// track.hip -- many-path tracking of gamma (1-t) g(x) + t f(x) = 0 from t = 0 to
// t = 1 (Section 2 of the paper, Tables 1-3), on one GPU: host side.  The
// device code (ph_track_dev.hpp) is compiled per residual precision and solve
// precision from track_unit.hip.
#include <hip/hip_runtime.h>

#include "ph_internal.hpp"
#include "ph_track.hpp"

namespace ph {

__global__ void clear_counter_kernel(unsigned int *c) { *c = 0u; }

int track_launch(const TrackArgs &a, int prec, int kmax, int blocks, size_t lds, hipStream_t st, int *occ)
{
    if (a.o.mixed) {
        switch (prec) {
        case 1: return track_launch_t<1, true>(a, kmax, blocks, lds, st, occ);
        case 2: return track_launch_t<2, true>(a, kmax, blocks, lds, st, occ);
        default: return track_launch_t<4, true>(a, kmax, blocks, lds, st, occ);
        }
    }
    switch (prec) {
    case 1: return track_launch_t<1, false>(a, kmax, blocks, lds, st, occ);
    case 2: return track_launch_t<2, false>(a, kmax, blocks, lds, st, occ);
    default: return track_launch_t<4, false>(a, kmax, blocks, lds, st, occ);
    }
}

size_t track_lds_bytes(int prec, int mixed, int np_max)
{
    const int ls = mixed ? 1 : prec;
    const size_t w = (size_t)(64 / np_max) * (np_max + 1) * np_max * 2 * ls;
    return (64 * 2 * (size_t)prec + w) * sizeof(double);
}

size_t slot_bytes(int prec)
{
    return prec == 1 ? slot_bytes_t<1>() : (prec == 2 ? slot_bytes_t<2>() : slot_bytes_t<4>());
}

int slot_init_launch(int prec, void *state, int64_t nslots, hipStream_t st)
{
    return prec == 1 ? slot_init_launch_t<1>(state, nslots, st)
                     : (prec == 2 ? slot_init_launch_t<2>(state, nslots, st) : slot_init_launch_t<4>(state, nslots, st));
}

int clear_counter_launch(unsigned int *c, hipStream_t st)
{
    hipLaunchKernelGGL(clear_counter_kernel, dim3(1), dim3(1), 0, st, c);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "clear_counter_kernel launch");
    return PH_OK;
}

}  // namespace ph

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

namespace ph {

static int check_opts(const ph_track_opts &o)
{
    if (o.prec != 1 && o.prec != 2 && o.prec != 4) return fail(PH_EINVAL, "opts.prec must be 1, 2 or 4");
    if (o.predictor_order < 1 || o.predictor_order > 4)
        return fail(PH_EUNSUPPORTED, "predictor_order must be 1 (secant) to 4");
    if (o.max_newton < 1 || o.expand_after < 1 || o.polish_max < 0 || o.max_steps < 0)
        return fail(PH_EINVAL, "invalid iteration counts in opts");
    if (!(o.h_init > 0) || !(o.h_max > 0) || !(o.h_min >= 0) || !(o.shrink > 0 && o.shrink < 1) ||
        !(o.expand >= 1) || !(o.tol_dx > 0) || !(o.diverge_norm > 0) || !(o.tol_res >= 0) ||
        !(o.launch_ms >= 0) || !(o.launch_ms <= 60000))
        return fail(PH_EINVAL, "invalid step-control constants in opts");
    if (o.lanes_per_path != 0 && o.lanes_per_path != 4 && o.lanes_per_path != 8 &&
        o.lanes_per_path != 16 && o.lanes_per_path != 32)
        return fail(PH_EINVAL, "lanes_per_path must be 0, 4, 8, 16 or 32");
    return PH_OK;
}

static double unit_roundoff(int prec)
{
    return prec == 1 ? std::ldexp(1.0, -53) : (prec == 2 ? std::ldexp(1.0, -104) : std::ldexp(1.0, -208));
}

static double eps_singular(int ls)
{
    return ls == 1 ? 1e-13 : (ls == 2 ? std::ldexp(1.0, -96) : std::ldexp(1.0, -200));
}

struct StreamGuard {
    hipStream_t s = nullptr;
    ~StreamGuard()
    {
        if (s) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
    }
};

struct DevBuf {
    void *p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
};

// Device scratch of the entry point for callers that cannot allocate
// (ph_track_noalloc): counters and work queues, the system descriptor and the
// predictor history of one call live in this file-scope array, one copy per
// GPU, held until the process ends.  Host code never passes the array's name
// to a kernel or a copy (on the host it is only a stand-in symbol); it uses
// the device address that hipGetSymbolAddress returns for the current device.
constexpr size_t NOALLOC_BYTES = size_t(16) << 20;
constexpr size_t NOALLOC_DESC_OFF = 4096;          // after the counters
constexpr size_t NOALLOC_HIST_OFF = size_t(64) << 10;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

struct NoallocScratch {
    void *ptr = nullptr;
    bool done = false;
};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
static int noalloc_scratch_ptr(void **out)
{
    static std::mutex mu;
    static NoallocScratch per_dev[64];
    int dev = 0;
    PH_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(PH_EUNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lk(mu);
    NoallocScratch &e = per_dev[dev];
    if (!e.done) {
        void *p = nullptr;
        hipError_t er = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (er != hipSuccess || !p) return hip_fail(er, "hipGetSymbolAddress(scratch)");
        e.ptr = p;
        e.done = true;
    }
    *out = e.ptr;
    return PH_OK;
}

// noalloc: device scratch for the no-allocation entry point (its address on
// the current device), or NULL to allocate per call.
static int track_impl(int nsys, const ph_system *const *targets, const ph_system *start,
                      const double *gammas, const int64_t *path_off, const int64_t *path_ids,
                      const double *x_start, int64_t ld, const ph_track_opts *opts, double *x_end,
                      int8_t *status, int8_t *reason, int32_t *steps, ph_track_report *rep,
                      hipStream_t st, unsigned char *noalloc = nullptr)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!opts) return fail(PH_EINVAL, "null opts");
    int rc = check_opts(*opts);
    if (rc) return rc;
    if (nsys < 1 || !targets || !gammas || !path_off) return fail(PH_EINVAL, "null batch arrays");
    const int64_t total = path_off[nsys];
    if (path_off[0] != 0) return fail(PH_EINVAL, "path_off[0] must be 0");
    for (int s = 0; s < nsys; ++s)
        if (path_off[s + 1] < path_off[s]) return fail(PH_EINVAL, "path_off not monotone");
    if (rep) *rep = ph_track_report{};
    if (total == 0) return PH_OK;
    if (!x_end || !status) return fail(PH_EINVAL, "null x_end or status");
    if (ld < total) return fail(PH_EINVAL, "ld < number of paths");
    const int prec = opts->prec;

    int dev = 0, cus = 256;
    PH_HIP(hipGetDevice(&dev));
    PH_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    // lanes per path: as asked, else the natural count, doubled when the
    // paths at their natural count fill less than one wave per SIMD (the
    // extra lanes share each equation's term sweeps; results are unchanged)
    int lanes_pp = opts->lanes_per_path;
    if (lanes_pp == 0) {
        double lanes = 0;
        int nat_max = 4;
        for (int s = 0; s < nsys; ++s) {
            if (!targets[s]) return fail(PH_EINVAL, "null target system");
            int nat = 4;
            while (nat < targets[s]->h.n_var) nat *= 2;
            nat_max = std::max(nat_max, nat);
            lanes += (double)(path_off[s + 1] - path_off[s]) * nat;
        }
        if (lanes < 64.0 * 4 * cus && 2 * nat_max <= 32) lanes_pp = 2 * nat_max;
    }

    // ---- systems grouped by lane-count class (4, 8, 16, 32 lanes per path)
    std::vector<SysDesc> desc;
    desc.reserve(nsys);
    TrackArgs a;
    std::memset(&a, 0, sizeof a);
    int kmax = 1, np_max = 4;
    const int class_np[4] = {4, 8, 16, 32};
    double work[4] = {0, 0, 0, 0};
    for (int c = 0; c < 4; ++c) {
        a.cls[c].np = class_np[c];
        a.cls[c].sys_first = (int)desc.size();
        int64_t q = 0;
        for (int s = 0; s < nsys; ++s) {
            const ph_system *t = targets[s];
            if (!t) return fail(PH_EINVAL, "null target system");
            const int n = t->h.n_var;
            if (t->h.n_eq != n) return fail(PH_EUNSUPPORTED, "tracking needs square systems");
            if (n > 32) return fail(PH_EUNSUPPORTED, "tracking is limited to n <= 32");
            int cls = 0;
            while (class_np[cls] < n || class_np[cls] < lanes_pp) ++cls;
            if (cls != c) continue;
            const DevTable *tab = nullptr;
            rc = noalloc ? find_table(t, start, &tab) : get_table(t, start, &tab);
            if (rc) return rc;
            SysDesc d;
            std::memset(&d, 0, sizeof d);
            d.eq_off = tab->eq_off;
            d.tdesc = tab->tdesc;
            d.fac = tab->fac;
            d.fac8 = tab->fac8;
            d.coef = tab->coef;
            d.path_off = path_off[s];
            d.npaths = path_off[s + 1] - path_off[s];
            d.qoff = q;
            q += d.npaths;
            d.gre = gammas[2 * s];
            d.gim = gammas[2 * s + 1];
            d.n = n;
            d.kmax = tab->kmax;
            d.path_ids = (const int64_t *)(intptr_t)(path_ids ? s + 1 : 0);  // patched below
            int64_t r = 1;
            bool overflow = false;
            for (int i = 0; i < 64; ++i) {
                d.deg[i] = i < n ? t->h.deg[i] : 1;
                d.radix[i] = overflow ? INT64_MAX : r;
                if (i < n) {
                    if (r > INT64_MAX / std::max(1, d.deg[i])) overflow = true;
                    else r *= d.deg[i];
                }
            }
            if (!x_start) {
                for (int i = 0; i < n; ++i) {
                    const int dg = t->h.deg[i];
                    if (dg < 1 || 12 % dg != 0 || dg == 12)
                        return fail(PH_EUNSUPPORTED, "in-kernel start solutions need degrees in {1,2,3,4,6}");
                }
                // every path number names a start solution: 0 <= id < Bezout number
                const int64_t bez = overflow ? INT64_MAX : r;
                if (path_ids) {
                    for (int64_t q2 = path_off[s]; q2 < path_off[s + 1]; ++q2)
                        if (path_ids[q2] < 0 || path_ids[q2] >= bez)
                            return fail(PH_EINVAL, "path id outside 0 .. Bezout number - 1");
                } else if (d.npaths > bez) {
                    return fail(PH_EINVAL, "more paths than start solutions");
                }
            }
            kmax = std::max(kmax, tab->kmax);
            // work estimate: lanes times terms per equation
            work[c] += (double)d.npaths * class_np[c] * (double)tab->n_terms / std::max(1, n);
            desc.push_back(d);
        }
        a.cls[c].sys_end = (int)desc.size();
        a.cls[c].total = q;
        if (q > 0) np_max = std::max(np_max, class_np[c]);
    }
    if (kmax > 8) return fail(PH_EUNSUPPORTED, "tracking supports terms with at most 8 factors");

    // ---- device buffers: descriptors, path ids, counters, slot state
    DevBuf bdesc, bids, bctr, bstate, bhist;
    if (noalloc) {
        if (path_ids) return fail(PH_EUNSUPPORTED, "no-allocation tracking takes no path id list");
        if (opts->schedule != PH_SCHED_PERSISTENT)
            return fail(PH_EUNSUPPORTED, "no-allocation tracking runs the persistent schedule only");
        if (sizeof(SysDesc) * desc.size() > NOALLOC_HIST_OFF - NOALLOC_DESC_OFF)
            return fail(PH_EINVAL, "no-allocation tracking: too many systems for the scratch buffer");
    }
    if (path_ids) {
        PH_HIP(hipMalloc(&bids.p, sizeof(int64_t) * total));
        PH_HIP(hipMemcpyAsync(bids.p, path_ids, sizeof(int64_t) * total, hipMemcpyHostToDevice, st));
        for (auto &d : desc) {
            const int s = (int)(intptr_t)d.path_ids - 1;
            d.path_ids = (const int64_t *)bids.p + path_off[s];
        }
    }
    void *desc_dev = nullptr;
    unsigned long long *ctr = nullptr;
    if (noalloc) {
        desc_dev = noalloc + NOALLOC_DESC_OFF;
        ctr = reinterpret_cast<unsigned long long *>(noalloc);
    } else {
        PH_HIP(hipMalloc(&bdesc.p, sizeof(SysDesc) * desc.size()));
        PH_HIP(hipMalloc(&bctr.p, sizeof(unsigned long long) * 32));
        desc_dev = bdesc.p;
        ctr = (unsigned long long *)bctr.p;
    }
    PH_HIP(hipMemcpyAsync(desc_dev, desc.data(), sizeof(SysDesc) * desc.size(), hipMemcpyHostToDevice, st));
    // counters, queues and the active count start at zero on every call (the
    // no-allocation scratch keeps the previous call's contents)
    PH_HIP(hipMemsetAsync(ctr, 0, sizeof(unsigned long long) * 32, st));

    a.sys = (const SysDesc *)desc_dev;
    a.nsys = (int)desc.size();
    a.x_start = x_start;
    a.ld_start = ld;
    a.x_end = x_end;
    a.ld_end = ld;
    a.status = status;
    a.reason = reason;
    a.steps = steps;
    a.stats = ctr;              // [0..2] totals, [3 + reason] counts
    a.active = (unsigned int *)(ctr + 20);
    a.o = *opts;
    a.polish_tol = opts->polish_tol < 0 ? 8.0 * unit_roundoff(prec) : opts->polish_tol;
    a.eps_sing = eps_singular(opts->mixed ? 1 : prec);

    // ---- blocks: per class proportional to its work, capped by residency:
    // no more workgroups than fit the CUs at once, so that every workgroup of
    // a launch starts with it (a round launch whose last workgroups waited
    // for the first ones to end would run twice its budget, mostly idle)
    const size_t lds = track_lds_bytes(prec, opts->mixed, np_max);
    int per_cu = opts->blocks_per_cu > 0 ? opts->blocks_per_cu : 8;
    {
        int occ = 0;
        rc = track_launch(a, prec, kmax, 0, lds, st, &occ);
        if (rc) return rc;
        if (occ > 0) per_cu = std::min(per_cu, occ);
    }
    int cap = cus * per_cu;
    if (const char *env = std::getenv("PH_TRACK_BLOCKS")) {
        const int e = std::atoi(env);
        if (e > 0) cap = std::min(cap, e);
    }
    // the shares are rounded down and then trimmed so that the classes
    // together never exceed the cap (one workgroup over it would start only
    // when a whole CU's worth had ended)
    double wsum = work[0] + work[1] + work[2] + work[3];
    int nbc[4] = {0, 0, 0, 0};
    int blocks = 0;
    for (int c = 0; c < 4; ++c) {
        if (a.cls[c].total > 0) {
            const int64_t need = (a.cls[c].total + (64 / class_np[c]) - 1) / (64 / class_np[c]);
            nbc[c] = (int)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)std::floor(cap * work[c] / wsum)));
        }
        blocks += nbc[c];
    }
    while (blocks > cap) {
        int big = 0;
        for (int c = 1; c < 4; ++c)
            if (nbc[c] > nbc[big]) big = c;
        if (nbc[big] <= 1) break;
        --nbc[big];
        --blocks;
    }
    blocks = 0;
    for (int c = 0; c < 4; ++c) {
        a.cls[c].queue = ctr + 10 + c;
        blocks += nbc[c];
        a.cls[c].block_end = blocks;
    }
    if (opts->predictor_order > 1) {
        // three older points per lane slot, kept across launches
        a.hist_ld = (int64_t)blocks * 64;
        const size_t hist_bytes = sizeof(double) * 3 * 2 * prec * (size_t)a.hist_ld;
        if (noalloc) {
            if (hist_bytes > NOALLOC_BYTES - NOALLOC_HIST_OFF) {
                char msg[200];
                std::snprintf(msg, sizeof msg,
                              "no-allocation tracking: the predictor history of %d workgroups needs %zu bytes, "
                              "more than the %zu of the scratch buffer (lower blocks_per_cu)",
                              blocks, hist_bytes, NOALLOC_BYTES - NOALLOC_HIST_OFF);
                return fail(PH_EINVAL, msg);
            }
            a.hist = reinterpret_cast<double *>(noalloc + NOALLOC_HIST_OFF);
        } else {
            PH_HIP(hipMalloc(&bhist.p, hist_bytes));
            a.hist = static_cast<double *>(bhist.p);
        }
    }

    if (opts->schedule == PH_SCHED_GRAPH) {
        // round-based: slot state in global memory, {clear, round kernel}
        // captured once and replayed; the host reads the number of waves
        // still active every launches_per_sync replays
        const int64_t nslots = (int64_t)blocks * 64;
        PH_HIP(hipMalloc(&bstate.p, slot_bytes(prec) * nslots));
        rc = slot_init_launch(prec, bstate.p, nslots, st);
        if (rc) return rc;
        a.state = bstate.p;
        a.rounds = std::max(1, opts->rounds_per_launch);
        if (opts->launch_ms > 0) {
            int khz = 0;  // wall clock of wall_clock64()
            PH_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
            if (khz <= 0) khz = 100000;
            a.budget = (unsigned long long)std::max(1.0, opts->launch_ms * khz);
            a.rounds = 0x7fffffff;
        }
        // capture and replay on a private stream (the legacy default stream
        // cannot be captured), ordered after the caller's stream
        StreamGuard cs;
        PH_HIP(hipStreamCreateWithFlags(&cs.s, hipStreamNonBlocking));
        hipEvent_t ready = nullptr;
        PH_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
        hipError_t er = hipEventRecord(ready, st);
        if (er == hipSuccess) er = hipStreamWaitEvent(cs.s, ready, 0);
        (void)hipEventDestroy(ready);
        if (er != hipSuccess) return hip_fail(er, "ordering the graph stream");
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        PH_HIP(hipStreamBeginCapture(cs.s, hipStreamCaptureModeThreadLocal));
        int rc1 = clear_counter_launch(a.active, cs.s);
        int rc2 = rc1 ? rc1 : track_launch(a, prec, kmax, blocks, lds, cs.s);
        hipError_t ec = hipStreamEndCapture(cs.s, &graph);
        if (rc2) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc2;
        }
        if (ec != hipSuccess) return hip_fail(ec, "hipStreamEndCapture");
        hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return hip_fail(ei, "hipGraphInstantiate");
        }
        const int sync_every = std::max(1, opts->launches_per_sync);
        const int64_t max_launches =
            (opts->max_steps + 2) * (int64_t)(opts->max_newton + 1) * 4 / a.rounds + 1000000;
        int64_t launches = 0;
        unsigned int active = 1;
        rc = PH_OK;
        while (active > 0 && launches < max_launches) {
            for (int k = 0; k < sync_every; ++k) {
                hipError_t e = hipGraphLaunch(exec, cs.s);
                if (e != hipSuccess) {
                    rc = hip_fail(e, "hipGraphLaunch");
                    break;
                }
                ++launches;
            }
            if (rc) break;
            hipError_t e = hipMemcpyAsync(&active, a.active, sizeof(unsigned int),
                                          hipMemcpyDeviceToHost, cs.s);
            if (e == hipSuccess) e = hipStreamSynchronize(cs.s);
            if (e != hipSuccess) {
                rc = hip_fail(e, "reading the active count");
                break;
            }
        }
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        if (rc) return rc;
        if (active > 0) return fail(PH_EHIP, "graph schedule did not drain the work queue");
    } else {
        a.state = nullptr;
        rc = track_launch(a, prec, kmax, blocks, lds, st);
        if (rc) return rc;
    }
    unsigned long long h[16];
    PH_HIP(hipMemcpyAsync(h, ctr, sizeof(h), hipMemcpyDeviceToHost, st));
    PH_HIP(hipStreamSynchronize(st));
    if (rep) {
        rep->steps = (int64_t)h[0];
        rep->rejected = (int64_t)h[1];
        rep->newton_its = (int64_t)h[2];
        const unsigned long long *c = h + 3;  // counts per reason
        rep->n_success = (int64_t)c[PH_R_SUCCESS];
        rep->n_diverged = (int64_t)c[PH_R_DIVERGED];
        rep->n_step_underflow = (int64_t)c[PH_R_STEP_UNDERFLOW];
        rep->n_max_steps = (int64_t)c[PH_R_MAX_STEPS];
        rep->n_singular = (int64_t)c[PH_R_SINGULAR];
        rep->n_nan = (int64_t)c[PH_R_NAN];
        rep->n_fail = total - rep->n_success;
        rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return PH_OK;
}

}  // namespace ph

using namespace ph;

extern "C" int ph_track(const ph_system *target, const ph_system *start, const double gamma[2],
                        int64_t npaths, const double *x_start, int64_t ld,
                        const ph_track_opts *opts, double *x_end, int8_t *status, int8_t *reason,
                        int32_t *steps, ph_track_report *rep, void *stream)
{
    if (!target || !gamma) return fail(PH_EINVAL, "null target or gamma");
    if (npaths < 0) return fail(PH_EINVAL, "npaths < 0");
    if (start && !x_start) return fail(PH_EINVAL, "a custom start system needs x_start");
    if (start && (start->h.n_eq != target->h.n_eq || start->h.n_var != target->h.n_var))
        return fail(PH_EINVAL, "start system shape differs from target");
    const int64_t off[2] = {0, npaths};
    return track_impl(1, &target, start, gamma, off, nullptr, x_start, ld, opts, x_end, status,
                      reason, steps, rep, (hipStream_t)stream);
}

extern "C" int ph_track_noalloc(const ph_system *target, const ph_system *start, const double gamma[2],
                                int64_t npaths, const double *x_start, int64_t ld,
                                const ph_track_opts *opts, double *x_end, int8_t *status,
                                int8_t *reason, int32_t *steps, ph_track_report *rep, void *stream)
{
    if (!target || !gamma) return fail(PH_EINVAL, "null target or gamma");
    if (npaths < 0) return fail(PH_EINVAL, "npaths < 0");
    if (start && !x_start) return fail(PH_EINVAL, "a custom start system needs x_start");
    if (start && (start->h.n_eq != target->h.n_eq || start->h.n_var != target->h.n_var))
        return fail(PH_EINVAL, "start system shape differs from target");
    void *scr = nullptr;
    int rc = noalloc_scratch_ptr(&scr);
    if (rc) return rc;
    const int64_t off[2] = {0, npaths};
    return track_impl(1, &target, start, gamma, off, nullptr, x_start, ld, opts, x_end, status,
                      reason, steps, rep, (hipStream_t)stream, static_cast<unsigned char *>(scr));
}

extern "C" int ph_track_batch(int32_t nsys, const ph_system *const *targets, const double *gammas,
                              const int64_t *path_off, const int64_t *path_ids,
                              const ph_track_opts *opts, double *x_end, int64_t ld, int8_t *status,
                              int8_t *reason, int32_t *steps, ph_track_report *rep, void *stream)
{
    return track_impl(nsys, targets, nullptr, gammas, path_off, path_ids, nullptr, ld, opts, x_end,
                      status, reason, steps, rep, (hipStream_t)stream);
}

// Autotuning of the tracker's launch shape on a proportional sample.
extern "C" int ph_track_autotune(int32_t nsys, const ph_system *const *targets, const double *gammas,
                                 const int64_t *path_off, const int64_t *path_ids,
                                 const ph_track_opts *opts, int64_t sample, ph_track_opts *tuned,
                                 double *best_seconds, void *stream)
{
    if (!opts || !tuned) return fail(PH_EINVAL, "null opts or tuned");
    int rc = check_opts(*opts);
    if (rc) return rc;
    if (nsys < 1 || !targets || !gammas || !path_off) return fail(PH_EINVAL, "null batch arrays");
    if (path_off[0] != 0) return fail(PH_EINVAL, "path_off[0] must be 0");
    for (int s = 0; s < nsys; ++s) {
        if (!targets[s]) return fail(PH_EINVAL, "null target system");
        if (path_off[s + 1] < path_off[s]) return fail(PH_EINVAL, "path_off not monotone");
    }
    const int64_t total = path_off[nsys];
    if (total == 0 || sample < 1) return fail(PH_EINVAL, "autotuning needs paths and sample >= 1");
    hipStream_t st = (hipStream_t)stream;
    if (best_seconds) *best_seconds = 0;

    // key: systems, their path counts, precision and mixed
    uint64_t key = 1469598103934665603ull;
    auto mix = [&key](uint64_t v) {
        for (int b = 0; b < 8; ++b) key = (key ^ ((v >> (8 * b)) & 0xff)) * 1099511628211ull;
    };
    for (int s = 0; s < nsys; ++s) {
        mix(targets[s]->h.fingerprint);
        mix((uint64_t)(path_off[s + 1] - path_off[s]));
    }
    mix((uint64_t)opts->prec);
    mix((uint64_t)opts->mixed);
    const char *cache = std::getenv("PH_AUTOTUNE_CACHE");
    if (cache) {
        if (FILE *f = std::fopen(cache, "r")) {
            char line[512], tag[16];
            unsigned long long k = 0;
            int sch = 0, rnd = 0, bpc = 0, lanes = 0;
            double lms = 0, sec = 0;
            bool found = false;
            ph_track_opts o = *opts;
            // one entry per line "track <key> <schedule> <rounds> <blocks per CU>
            // <lanes> <launch ms> <seconds>"; lines of other tags are skipped
            while (std::fgets(line, sizeof line, f)) {
                if (std::sscanf(line, "%15s %llx %d %d %d %d %lf %lf", tag, &k, &sch, &rnd, &bpc, &lanes, &lms,
                                &sec) == 8 &&
                    std::strcmp(tag, "track") == 0 && k == key) {
                    o.schedule = sch;
                    o.rounds_per_launch = rnd;
                    o.blocks_per_cu = bpc;
                    o.lanes_per_path = lanes;
                    o.launch_ms = lms;
                    found = true;
                }
            }
            std::fclose(f);
            if (found) {
                *tuned = o;
                return PH_OK;
            }
        }
    }

    // proportional sample: each system's first paths (or first listed ids)
    const double frac = std::min(1.0, (double)sample / (double)total);
    std::vector<int64_t> off(nsys + 1, 0), ids;
    for (int s = 0; s < nsys; ++s) {
        const int64_t np = path_off[s + 1] - path_off[s];
        const int64_t m = np == 0 ? 0 : std::max<int64_t>(1, (int64_t)std::ceil(np * frac));
        for (int64_t p = 0; p < m; ++p) ids.push_back(path_ids ? path_ids[path_off[s] + p] : p);
        off[s + 1] = off[s] + m;
    }
    const int64_t ns = off[nsys];
    int maxn = 1;
    for (int s = 0; s < nsys; ++s) maxn = std::max(maxn, (int)targets[s]->h.n_var);
    DevBuf bx, bst;
    PH_HIP(hipMalloc(&bx.p, sizeof(double) * (size_t)maxn * 2 * opts->prec * ns));
    PH_HIP(hipMalloc(&bst.p, (size_t)ns));

    // candidates: residency-limited workgroups per CU, both schedules, the
    // natural lane count and two or four times it (the extra lanes share each
    // equation's term sweeps: more waves and shorter rounds for few paths)
    int np_max = 4;
    while (np_max < maxn) np_max *= 2;
    // (graph schedule: fixed round counts and time budgets per launch)
    struct Cand { int sch, rnd, bpc, lanes; double lms; };
    std::vector<Cand> cands;
    for (int lanes : {0, 2 * np_max, 4 * np_max}) {
        if (lanes > 32) continue;
        const int lcap = (int)std::max<size_t>(
            1, (160 * 1024) / track_lds_bytes(opts->prec, opts->mixed, lanes ? lanes : np_max));
        for (int bpc : {2, 4, 8, 12, 16})
            if (bpc <= lcap || bpc == 2)
                cands.push_back({PH_SCHED_PERSISTENT, opts->rounds_per_launch, bpc, lanes, opts->launch_ms});
        for (int rnd : {8, 32, 128}) cands.push_back({PH_SCHED_GRAPH, rnd, std::min(8, lcap), lanes, 0.0});
        for (double lms : {1.0, 2.0, 4.0}) cands.push_back({PH_SCHED_GRAPH, 32, std::min(8, lcap), lanes, lms});
    }
    double best = 1e300;
    ph_track_opts bo = *opts;
    for (const Cand &c : cands) {
        ph_track_opts o = *opts;
        o.schedule = c.sch;
        o.rounds_per_launch = c.rnd;
        o.blocks_per_cu = c.bpc;
        o.lanes_per_path = c.lanes;
        o.launch_ms = c.lms;
        ph_track_report r;
        rc = track_impl(nsys, targets, nullptr, gammas, off.data(), ids.data(), nullptr, ns, &o,
                        (double *)bx.p, (int8_t *)bst.p, nullptr, nullptr, &r, st);
        if (rc) return rc;
        if (r.seconds < best) {
            best = r.seconds;
            bo = o;
        }
    }
    *tuned = bo;
    if (best_seconds) *best_seconds = best;
    if (cache) {
        if (FILE *f = std::fopen(cache, "a")) {
            std::fprintf(f, "track %llx %d %d %d %d %.3f %.6f\n", (unsigned long long)key, bo.schedule,
                         bo.rounds_per_launch, bo.blocks_per_cu, bo.lanes_per_path, bo.launch_ms, best);
            std::fclose(f);
        }
    }
    return PH_OK;
}
