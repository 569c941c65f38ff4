// track.hip -- many-path tracking of gamma (1-t) g(x) + t f(x) = 0 from t = 0 to
// t = 1 (Section 2 of the paper, Tables 1-3), on one GPU.
//
// Mapping onto gfx950:
//   * a path occupies NP consecutive lanes of a wave (NP = power of two >= n);
//     lane i of the group owns coordinate i of the point and row i of H and J,
//     so evaluation produces the Jacobian directly in the row layout the
//     least-squares solve consumes (the paper transposes the Jacobian between
//     the evaluate and correct kernels, Section 3);
//   * the augmented matrix [J | -H] of every path lives in LDS, column-major
//     with the row index fastest, and is reduced by modified Gram-Schmidt with
//     group butterflies (shuffles) for the column norms and inner products;
//   * the kernel is persistent: every group pops path indices from one device
//     counter and refills itself when its path ends (Table 2's relabeling of
//     finished paths becomes a refill; Table 3's scan is not needed because no
//     host round trip happens at all);
//   * each round performs one Newton iteration (evaluate + correct) for every
//     occupied group, so the expensive parts never diverge; predicting,
//     accepting, rejecting, step-size control, status and polishing are cheap
//     per-path decisions taken between rounds (Table 1: paths need different
//     numbers of evaluate-correct stages);
//   * mixed precision: the residual and the Jacobian are evaluated in L limbs;
//     the Jacobian partials and the residual are rounded to FP64, the update is
//     solved in FP64 and added to the L-limb point (iterative refinement).
//     Plain mode solves in L limbs.
#include <hip/hip_runtime.h>

#include "ph_arith.hpp"
#include "ph_internal.hpp"
#include "ph_sweep.hpp"
#include "ph_track.hpp"

namespace ph {

template <int NP>
__device__ __forceinline__ double gsum_d(double v)
{
#pragma unroll
    for (int o = 1; o < NP; o <<= 1) v += __shfl_xor(v, o);
    return v;
}

template <int NP>
__device__ __forceinline__ double gmax_d(double v)
{
#pragma unroll
    for (int o = 1; o < NP; o <<= 1) {
        double u = __shfl_xor(v, o);
        v = (v != v || u != u) ? (v + u) : fmax(v, u);  // NaN propagates
    }
    return v;
}

template <int NP, int L>
__device__ __forceinline__ R<L> gsum_r(R<L> v)
{
#pragma unroll
    for (int o = 1; o < NP; o <<= 1) {
        R<L> u;
#pragma unroll
        for (int l = 0; l < L; ++l) u.v[l] = __shfl_xor(v.v[l], o);
        v = r_add<L>(v, u);
    }
    return v;
}

template <int NP, int L>
__device__ __forceinline__ C<L> gsum_c(C<L> v)
{
    return C<L>{gsum_r<NP, L>(v.re), gsum_r<NP, L>(v.im)};
}

template <int L>
__device__ __forceinline__ C<L> shfl_c(C<L> v, int src)
{
    C<L> r;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        r.re.v[l] = __shfl(v.re.v[l], src);
        r.im.v[l] = __shfl(v.im.v[l], src);
    }
    return r;
}

template <int L>
__device__ __forceinline__ double c_absd(C<L> a)
{
    return hypot(a.re.v[0], a.im.v[0]);
}

template <int L>
__device__ __forceinline__ bool c_bad(C<L> a)
{
    return !isfinite(a.re.v[0]) || !isfinite(a.im.v[0]);
}

// LDS element access: 2 * LS doubles per complex entry.
template <int LS>
__device__ __forceinline__ C<LS> lds_get(const double *p)
{
    C<LS> z;
#pragma unroll
    for (int l = 0; l < LS; ++l) {
        z.re.v[l] = p[l];
        z.im.v[l] = p[LS + l];
    }
    return z;
}

template <int LS>
__device__ __forceinline__ void lds_put(double *p, C<LS> z)
{
#pragma unroll
    for (int l = 0; l < LS; ++l) {
        p[l] = z.re.v[l];
        p[LS + l] = z.im.v[l];
    }
}

template <int LS, int L>
__device__ __forceinline__ C<LS> narrow(C<L> a)
{
    C<LS> r = c_zero<LS>();
#pragma unroll
    for (int l = 0; l < LS; ++l) {
        r.re.v[l] = a.re.v[l];
        r.im.v[l] = a.im.v[l];
    }
    return r;
}

template <int L, int LS>
__device__ __forceinline__ C<L> widen_add(C<L> a, C<LS> d)
{
    if constexpr (LS == L) {
        return c_add<L>(a, d);
    } else {
        return c_add_c64<L>(a, d.re.v[0], d.im.v[0]);
    }
}

// Root of unity exp(2 pi i k / d) for d dividing 12, in L limbs.
template <int L>
__device__ C<L> root_of_unity(int d, int k, const R<L> &h3)
{
    const int a = ((12 / d) * (k % d)) % 12;
    R<L> c = r_zero<L>(), s = r_zero<L>();
    switch (a) {
    case 0: c = r_from<L>(1.0); break;
    case 2: c = r_from<L>(0.5); s = h3; break;
    case 3: s = r_from<L>(1.0); break;
    case 4: c = r_from<L>(-0.5); s = h3; break;
    case 6: c = r_from<L>(-1.0); break;
    case 8: c = r_from<L>(-0.5); s = r_neg<L>(h3); break;
    case 9: s = r_from<L>(-1.0); break;
    case 10: c = r_from<L>(0.5); s = r_neg<L>(h3); break;
    default: break;
    }
    return C<L>{c, s};
}

template <int L>
__device__ R<L> half_sqrt3_t()
{
    R<L> three = r_from<L>(3.0);
    return r_mul_d<L>(r_sqrt<L>(three), 0.5);
}

enum : int { PH_EMPTY = 0, PH_STEP = 1, PH_CORRECT = 2, PH_POLISH = 3, PH_RETIRED = 4 };

template <int L, int NP, int KMAX, bool MIXED>
__global__ void __launch_bounds__(64) track_kernel(TrackArgs a)
{
    constexpr int PPW = 64 / NP;
    constexpr int LS = MIXED ? 1 : L;
    __shared__ double xsh[PPW][NP][2 * L];
    __shared__ double wsh[PPW][NP + 1][NP][2 * LS];

    const int lane = threadIdx.x;
    const int g = lane / NP;
    const int i = lane % NP;
    const int base = g * NP;
    const ph_track_opts &o = a.o;
    const R<L> h3 = half_sqrt3_t<L>();

    // per-slot state, identical in every lane of a group
    int phase = PH_EMPTY;
    int64_t gid = 0, pid = 0;
    int sidx = 0, n = 0;
    double t = 0, tp = 0, t1 = 0, h = 0, dprev = 0;
    int succ = 0, it = 0, have_prev = 0, pit = 0;
    int32_t steps = 0, rejected = 0, newton = 0;
    // per-lane coordinate i
    C<L> x = c_zero<L>(), xp = c_zero<L>(), xh = c_zero<L>();

    auto finish = [&](int reason) {
        if (i < n) {
#pragma unroll
            for (int l = 0; l < L; ++l) {
                a.x_end[((int64_t)(i * 2 + 0) * L + l) * a.ld_end + gid] = x.re.v[l];
                a.x_end[((int64_t)(i * 2 + 1) * L + l) * a.ld_end + gid] = x.im.v[l];
            }
        }
        if (i == 0) {
            a.status[gid] = reason == PH_R_SUCCESS ? 1 : -1;
            if (a.reason) a.reason[gid] = (int8_t)reason;
            if (a.steps) a.steps[gid] = steps;
            if (a.newton) a.newton[gid] = newton;
            atomicAdd(&a.stats[0], (unsigned long long)steps);
            atomicAdd(&a.stats[1], (unsigned long long)rejected);
            atomicAdd(&a.stats[2], (unsigned long long)newton);
            atomicAdd(&a.stats[3 + reason], 1ull);
        }
        phase = PH_EMPTY;
        n = 0;
    };

    for (;;) {
        // ---- refill: pop a path from the device queue --------------------
        if (phase == PH_EMPTY) {
            unsigned long long id = 0;
            if (i == 0) id = atomicAdd(a.queue, 1ull);
            id = __shfl(id, base);
            if ((int64_t)id >= a.total_paths) {
                phase = PH_RETIRED;
                n = 0;
            } else {
                gid = (int64_t)id;
                sidx = 0;
                while (sidx + 1 < a.nsys && a.sys[sidx + 1].path_off <= gid) ++sidx;
                const SysDesc &sd = a.sys[sidx];
                n = sd.n;
                const int64_t local = gid - sd.path_off;
                pid = sd.path_ids ? sd.path_ids[local] : local;
                x = c_zero<L>();
                if (i < n) {
                    if (a.x_start) {
#pragma unroll
                        for (int l = 0; l < L; ++l) {
                            x.re.v[l] = a.x_start[((int64_t)(i * 2 + 0) * L + l) * a.ld_start + gid];
                            x.im.v[l] = a.x_start[((int64_t)(i * 2 + 1) * L + l) * a.ld_start + gid];
                        }
                    } else {
                        const int d = sd.deg[i];
                        const int k = (int)((pid / sd.radix[i]) % d);
                        x = root_of_unity<L>(d, k, h3);
                    }
                }
                xp = x;
                xh = x;
                t = tp = 0.0;
                h = o.h_init;
                succ = it = have_prev = pit = 0;
                steps = rejected = newton = 0;
                phase = PH_STEP;
            }
        }
        const bool any_bad = gmax_d<NP>(c_bad<L>(x) ? 1.0 : 0.0) > 0.0;
        if (phase == PH_STEP && steps == 0) {
            if (o.h_min > o.h_init) finish(PH_R_STEP_UNDERFLOW);
            else if (any_bad) finish(PH_R_NAN);
        }
        // ---- exit when every slot of the wave is retired -----------------
        if (__all(phase == PH_RETIRED)) break;

        // ---- predictor ----------------------------------------------------
        if (phase == PH_STEP) {
            if (steps >= o.max_steps) {
                finish(PH_R_MAX_STEPS);
            } else {
                ++steps;
                if (h > 1.0 - t) h = 1.0 - t;
                t1 = t + h;
                if (t1 >= 1.0 - 1e-15) t1 = 1.0;
                if (have_prev) {
                    const double r = (t1 - t) / (t - tp);
                    xh = c_add<L>(x, c_mul_d<L>(c_sub<L>(x, xp), r));
                } else {
                    xh = x;
                }
                it = 0;
                dprev = 0.0;
                phase = PH_CORRECT;
            }
        }
        const bool busy = phase == PH_CORRECT || phase == PH_POLISH;
        const double tt = phase == PH_POLISH ? 1.0 : t1;
        const SysDesc &sd = a.sys[sidx];

        // ---- evaluate H and J at (xh, tt): lane i does equation i ----------
        double *xg = &xsh[g][0][0];
#pragma unroll
        for (int l = 0; l < L; ++l) {
            xsh[g][i][l] = xh.re.v[l];
            xsh[g][i][L + l] = xh.im.v[l];
        }
#pragma unroll
        for (int j = 0; j <= NP; ++j) lds_put<LS>(&wsh[g][j][i][0], c_zero<LS>());
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        C<L> v = c_zero<L>();
        if (busy && i < n) {
            double o1, oe;
            two_sum(1.0, -tt, o1, oe);
            R<L> omt = r_zero<L>();
            omt.v[0] = o1;
            if constexpr (L > 1) omt.v[1] = oe;
            const C<L> gs = c_mul_r<L>(c_from<L>(sd.gre, sd.gim), omt);
            auto X = [&](int var) -> C<L> {
                C<L> z;
#pragma unroll
                for (int l = 0; l < L; ++l) {
                    z.re.v[l] = xg[var * 2 * L + l];
                    z.im.v[l] = xg[var * 2 * L + L + l];
                }
                return z;
            };
            const int s0 = sd.eq_off[i], s1 = sd.eq_off[i + 1];
            for (int s = s0; s < s1; ++s) {
                const int4 d = sd.tdesc[s];
                C<L> c;
#pragma unroll
                for (int l = 0; l < L; ++l) {
                    c.re.v[l] = sd.coef[(int64_t)s * 8 + l];
                    c.im.v[l] = sd.coef[(int64_t)s * 8 + 4 + l];
                }
                c = d.z ? c_mul<L>(c, gs) : c_mul_d<L>(c, tt);
                if (d.x == 0) {
                    v = c_add<L>(v, c);
                    continue;
                }
                uint32_t fw[KMAX];
#pragma unroll
                for (int l = 0; l < KMAX; ++l)
                    if (l < d.x) fw[l] = sd.fac[d.y + l];
                v = c_add<L>(v, term_sweep<KMAX, true>(
                                    d.x, fw, c, X, [&](int, uint32_t w, const C<L> &part) {
                                        double *e = &wsh[g][fac_var(w)][i][0];
                                        lds_put<LS>(e, c_add<LS>(lds_get<LS>(e), narrow<LS, L>(part)));
                                    }));
            }
            lds_put<LS>(&wsh[g][NP][i][0], narrow<LS, L>(c_sub<L>(c_zero<L>(), v)));
        }

        // ---- correct: MGS least squares on [J | -H], row i in lane i ------
        // Frobenius norm of J for the rank test
        double fro = 0.0;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            C<LS> w = lds_get<LS>(&wsh[g][j][i][0]);
            fro += w.re.v[0] * w.re.v[0] + w.im.v[0] * w.im.v[0];
        }
        fro = sqrt(gsum_d<NP>(fro));
        bool sing = false;
        C<LS> acc = c_zero<LS>();  // r_{i,rhs} then back-substituted value
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            if (k < n) {  // group-uniform
                C<LS> wk = lds_get<LS>(&wsh[g][k][i][0]);
                R<LS> nr = gsum_r<NP, LS>(c_abs2<LS>(wk));
                R<LS> rkk = r_sqrt<LS>(nr);
                if (!(rkk.v[0] > a.eps_sing * fro)) sing = true;
                if (!sing) {
                    R<LS> inv = r_div<LS>(r_from<LS>(1.0), rkk);
                    C<LS> q = c_mul_r<LS>(wk, inv);
#pragma unroll
                    for (int j = k + 1; j <= NP; ++j) {
                        if (j < n || j == NP) {
                            double *ej = &wsh[g][j][i][0];
                            C<LS> wj = lds_get<LS>(ej);
                            C<LS> r = gsum_c<NP, LS>(c_cmul<LS>(q, wj));
                            lds_put<LS>(ej, c_sub<LS>(wj, c_mul<LS>(r, q)));
                            // R row k is kept in the dead column k: entry (k, j) at row j
                            if (i == k) {
                                if (j == NP) acc = r;
                            }
                            if (j < NP) {
                                // lane j stores r_kj into column k, row j (column k is dead after step k)
                                C<LS> rr = r;
                                if (i == j) lds_put<LS>(&wsh[g][k][j][0], rr);
                            }
                        }
                    }
                    if (i == k) lds_put<LS>(&wsh[g][k][k][0], C<LS>{rkk, r_zero<LS>()});
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        // back substitution R dx = r_rhs, column oriented: lane i keeps acc_i
        C<LS> dxi = c_zero<LS>();
#pragma unroll
        for (int k = NP - 1; k >= 0; --k) {
            if (k < n && !sing) {
                C<LS> dk = c_zero<LS>();
                if (i == k) {
                    R<LS> rkk = lds_get<LS>(&wsh[g][k][k][0]).re;
                    R<LS> inv = r_div<LS>(r_from<LS>(1.0), rkk);
                    dk = c_mul_r<LS>(acc, inv);
                    dxi = dk;
                }
                dk = shfl_c<LS>(dk, base + k);
                if (i < k) {
                    C<LS> rik = lds_get<LS>(&wsh[g][i][k][0]);  // R(i, k) stored at column i, row k
                    acc = c_sub<LS>(acc, c_mul<LS>(rik, dk));
                }
            }
        }
        // rows >= n and idle groups carry zeros
        if (i >= n || !busy) dxi = c_zero<LS>();

        // ---- per-path decisions ------------------------------------------
        if (phase == PH_CORRECT) {
            ++newton;
            bool accept = false, reject = false;
            if (sing) {
                reject = true;
            } else {
                xh = widen_add<L, LS>(xh, dxi);
                const double dn = gmax_d<NP>(i < n ? c_absd<LS>(dxi) : 0.0);
                const double xn = gmax_d<NP>(i < n ? c_absd<L>(xh) : 0.0);
                if (dn != dn || xn != xn) {
                    reject = true;
                } else if (dn <= o.tol_dx * (xn > 1.0 ? xn : 1.0)) {
                    accept = true;
                } else if (it >= 1 && dn > dprev) {
                    reject = true;
                } else {
                    dprev = dn;
                    ++it;
                    if (it >= o.max_newton) reject = true;
                }
            }
            if (accept) {
                tp = t;
                xp = x;
                have_prev = 1;
                t = t1;
                x = xh;
                if (++succ >= o.expand_after) {
                    h = h * o.expand;
                    if (h > o.h_max) h = o.h_max;
                    succ = 0;
                }
                phase = (t == 1.0) ? PH_POLISH : PH_STEP;
                pit = 0;
                dprev = INFINITY;
            } else if (reject) {
                ++rejected;
                h *= o.shrink;
                succ = 0;
                phase = PH_STEP;
                if (h < o.h_min) finish(sing ? PH_R_SINGULAR : PH_R_STEP_UNDERFLOW);
            }
            if (accept || reject) {
                if (phase != PH_EMPTY) {
                    const bool bad = gmax_d<NP>((i < n && c_bad<L>(x)) ? 1.0 : 0.0) > 0.0;
                    const double xn = gmax_d<NP>(i < n ? c_absd<L>(x) : 0.0);
                    if (bad) finish(PH_R_NAN);
                    else if (xn > o.diverge_norm) finish(PH_R_DIVERGED);
                }
            }
        } else if (phase == PH_POLISH) {
            // Newton on f at t = 1 until the update meets polish_tol, stops
            // halving, or polish_max steps were taken
            bool done = false;
            if (sing) {
                done = true;
            } else {
                const double dn = gmax_d<NP>(i < n ? c_absd<LS>(dxi) : 0.0);
                if (pit > 0 && !(dn < 0.5 * dprev)) {
                    done = true;
                } else {
                    x = widen_add<L, LS>(x, dxi);
                    ++newton;
                    const double xn = gmax_d<NP>(i < n ? c_absd<L>(x) : 0.0);
                    if (dn <= a.polish_tol * (xn > 1.0 ? xn : 1.0)) done = true;
                    dprev = dn;
                    ++pit;
                    if (pit >= o.polish_max) done = true;
                }
            }
            xh = x;
            if (done) finish(PH_R_SUCCESS);
        }
    }
}

template <int L, int NP, bool MIXED>
static int launch_np(const TrackArgs &a, int kmax, int blocks, hipStream_t st)
{
    if (kmax <= 4) {
        hipLaunchKernelGGL((track_kernel<L, NP, 4, MIXED>), dim3(blocks), dim3(64), 0, st, a);
    } else {
        hipLaunchKernelGGL((track_kernel<L, NP, 8, MIXED>), dim3(blocks), dim3(64), 0, st, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "track_kernel launch");
    return PH_OK;
}

template <int L, bool MIXED>
static int launch_l(const TrackArgs &a, int np, int kmax, int blocks, hipStream_t st)
{
    switch (np) {
    case 4: return launch_np<L, 4, MIXED>(a, kmax, blocks, st);
    case 8: return launch_np<L, 8, MIXED>(a, kmax, blocks, st);
    case 16: return launch_np<L, 16, MIXED>(a, kmax, blocks, st);
    default: return launch_np<L, 32, MIXED>(a, kmax, blocks, st);
    }
}

int track_launch(const TrackArgs &a, int prec, int np, int kmax, int blocks, hipStream_t st)
{
    if (a.o.mixed) {
        switch (prec) {
        case 1: return launch_l<1, true>(a, np, kmax, blocks, st);
        case 2: return launch_l<2, true>(a, np, kmax, blocks, st);
        default: return launch_l<4, true>(a, np, kmax, blocks, st);
        }
    }
    switch (prec) {
    case 1: return launch_l<1, false>(a, np, kmax, blocks, st);
    case 2: return launch_l<2, false>(a, np, kmax, blocks, st);
    default: return launch_l<4, false>(a, np, kmax, blocks, st);
    }
}

}  // namespace ph

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <vector>

namespace ph {

static int check_opts(const ph_track_opts &o)
{
    if (o.prec != 1 && o.prec != 2 && o.prec != 4) return fail(PH_EINVAL, "opts.prec must be 1, 2 or 4");
    if (o.predictor_order != 1)
        return fail(PH_EUNSUPPORTED, "only the secant predictor (order 1) is implemented");
    if (o.max_newton < 1 || o.expand_after < 1 || o.polish_max < 0 || o.max_steps < 0)
        return fail(PH_EINVAL, "invalid iteration counts in opts");
    if (!(o.h_init > 0) || !(o.h_max > 0) || !(o.h_min >= 0) || !(o.shrink > 0 && o.shrink < 1) ||
        !(o.expand >= 1) || !(o.tol_dx > 0) || !(o.diverge_norm > 0))
        return fail(PH_EINVAL, "invalid step-control constants in opts");
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

struct DevBuf {
    void *p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
};

static int track_impl(int nsys, const ph_system *const *targets, const ph_system *start,
                      const double *gammas, const int64_t *path_off, const int64_t *path_ids,
                      const double *x_start, int64_t ld, const ph_track_opts *opts, double *x_end,
                      int8_t *status, int8_t *reason, int32_t *steps, ph_track_report *rep,
                      hipStream_t st)
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
    int nmax = 1, kmax = 1;
    std::vector<SysDesc> desc(nsys);
    for (int s = 0; s < nsys; ++s) {
        const ph_system *t = targets[s];
        if (!t) return fail(PH_EINVAL, "null target system");
        const int n = t->h.n_var;
        if (t->h.n_eq != n) return fail(PH_EUNSUPPORTED, "tracking needs square systems");
        if (n > 32) return fail(PH_EUNSUPPORTED, "tracking is limited to n <= 32");
        const DevTable *tab = nullptr;
        rc = get_table(t, start, &tab);
        if (rc) return rc;
        SysDesc &d = desc[s];
        d = SysDesc{};
        d.eq_off = tab->eq_off;
        d.tdesc = tab->tdesc;
        d.fac = tab->fac;
        d.coef = tab->coef;
        d.path_off = path_off[s];
        d.npaths = path_off[s + 1] - path_off[s];
        d.gre = gammas[2 * s];
        d.gim = gammas[2 * s + 1];
        d.n = n;
        d.kmax = tab->kmax;
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
        }
        nmax = std::max(nmax, n);
        kmax = std::max(kmax, tab->kmax);
    }
    if (kmax > 8) return fail(PH_EUNSUPPORTED, "tracking supports terms with at most 8 factors");
    int np = 4;
    while (np < nmax) np *= 2;

    // device buffers: descriptors, path ids, counters
    DevBuf bdesc, bids, bctr;
    PH_HIP(hipMalloc(&bdesc.p, sizeof(SysDesc) * nsys));
    if (path_ids) {
        PH_HIP(hipMalloc(&bids.p, sizeof(int64_t) * total));
        PH_HIP(hipMemcpyAsync(bids.p, path_ids, sizeof(int64_t) * total, hipMemcpyHostToDevice, st));
        for (int s = 0; s < nsys; ++s) desc[s].path_ids = (const int64_t *)bids.p + path_off[s];
    }
    PH_HIP(hipMemcpyAsync(bdesc.p, desc.data(), sizeof(SysDesc) * nsys, hipMemcpyHostToDevice, st));
    PH_HIP(hipMalloc(&bctr.p, sizeof(unsigned long long) * 16));
    PH_HIP(hipMemsetAsync(bctr.p, 0, sizeof(unsigned long long) * 16, st));

    TrackArgs a;
    a.sys = (const SysDesc *)bdesc.p;
    a.nsys = nsys;
    a.total_paths = total;
    a.x_start = x_start;
    a.ld_start = ld;
    a.x_end = x_end;
    a.ld_end = ld;
    a.status = status;
    a.reason = reason;
    a.steps = steps;
    a.newton = nullptr;
    a.queue = (unsigned long long *)bctr.p;
    a.stats = (unsigned long long *)bctr.p + 1;
    a.o = *opts;
    a.polish_tol = opts->polish_tol < 0 ? 8.0 * unit_roundoff(prec) : opts->polish_tol;
    a.eps_sing = eps_singular(opts->mixed ? 1 : prec);

    int dev = 0, cus = 256;
    PH_HIP(hipGetDevice(&dev));
    PH_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int ppw = 64 / np;
    const int64_t need = (total + ppw - 1) / ppw;
    int blocks = (int)std::min<int64_t>(need, (int64_t)cus * 16);
    // PH_TRACK_BLOCKS caps the number of persistent workgroups (a schedule
    // knob: results must not depend on it)
    if (const char *env = std::getenv("PH_TRACK_BLOCKS")) {
        const int cap = std::atoi(env);
        if (cap > 0) blocks = std::min(blocks, cap);
    }
    rc = track_launch(a, prec, np, kmax, blocks, st);
    if (rc) return rc;
    unsigned long long h[16];
    PH_HIP(hipMemcpyAsync(h, bctr.p, sizeof(h), hipMemcpyDeviceToHost, st));
    PH_HIP(hipStreamSynchronize(st));
    if (rep) {
        rep->steps = (int64_t)h[1];
        rep->rejected = (int64_t)h[2];
        rep->newton_its = (int64_t)h[3];
        const unsigned long long *c = h + 4;  // counts per reason
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

extern "C" int ph_track_batch(int32_t nsys, const ph_system *const *targets, const double *gammas,
                              const int64_t *path_off, const int64_t *path_ids,
                              const ph_track_opts *opts, double *x_end, int64_t ld, int8_t *status,
                              int8_t *reason, int32_t *steps, ph_track_report *rep, void *stream)
{
    return track_impl(nsys, targets, nullptr, gammas, path_off, path_ids, nullptr, ld, opts, x_end,
                      status, reason, steps, rep, (hipStream_t)stream);
}
