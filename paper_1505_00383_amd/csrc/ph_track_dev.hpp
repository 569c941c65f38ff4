// ph_track_dev.hpp -- device code of the path tracker (included by the
// per-precision translation units track_l1.hip, track_l2.hip, track_l4.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "ph_arith.hpp"
#include "ph_internal.hpp"
#include "ph_sweep.hpp"
#include "ph_track.hpp"

namespace ph {

// Partner value for step O (1, 2, 4, 8, 16) of a group reduction.  The
// first four steps stay inside a 16-lane row and use DPP moves (quad
// permutations, then the half-row and row mirrors, which pair each lane
// with one in the other half of its 8- or 16-lane block, as a reduction
// needs); the step across rows uses a lane permute.  After every step all
// lanes of a block hold bitwise the same value, because each pair adds the
// same two operands.  Every lane has a source lane in these permutations,
// so the DPP moves carry no "old" operand (which would cost a register set to
// zero per move).
template <int O>
__device__ __forceinline__ double red_partner(double v)
{
    if constexpr (O >= 16) {
        return __shfl_xor(v, O);
    } else {
        constexpr int ctrl = O == 1 ? 0xB1 : (O == 2 ? 0x4E : (O == 4 ? 0x141 : 0x140));
        const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
        const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, ctrl, 0xF, 0xF, true);
        const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), ctrl, 0xF, 0xF, true);
        return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
    }
}

template <int NP, int O = 1>
__device__ __forceinline__ double gsum_d(double v)
{
    if constexpr (O < NP) {
        v += red_partner<O>(v);
        return gsum_d<NP, 2 * O>(v);
    } else {
        return v;
    }
}

template <int NP, int O = 1>
__device__ __forceinline__ double gmax_d(double v)
{
    if constexpr (O < NP) {
        const double u = red_partner<O>(v);
        v = (v != v || u != u) ? (v + u) : fmax(v, u);  // NaN propagates
        return gmax_d<NP, 2 * O>(v);
    } else {
        return v;
    }
}

// L-limb sum over the group.  A zero operand is skipped rather than added:
// a multi-limb addition may renormalise the limbs of the other operand, and
// the rows and lanes a group has beyond its system's unknowns (zeros) must
// not change any bit of the result, whatever the lane count.
template <int NP, int L, int O = 1>
__device__ __forceinline__ R<L> gsum_r(R<L> v)
{
    if constexpr (O < NP) {
        R<L> u;
#pragma unroll
        for (int l = 0; l < L; ++l) u.v[l] = red_partner<O>(v.v[l]);
        R<L> s;
        if constexpr (L == 1) {
            s = r_add<L>(v, u);
        } else {
            s = u.v[0] == 0.0 ? v : (v.v[0] == 0.0 ? u : r_add<L>(v, u));
        }
        return gsum_r<NP, L, 2 * O>(s);
    } else {
        return v;
    }
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

// The value of the one lane of each group for which `mine` holds, in every
// lane of the group: the others contribute zero bits and the group ORs the
// bit patterns with the reduction's partner moves (DPP within a 16-lane
// row), so the value arrives bit for bit without a trip through LDS.
template <int NP, int O = 1>
__device__ __forceinline__ unsigned long long gbcast_bits(unsigned long long b)
{
    if constexpr (O < NP) {
        const double p = red_partner<O>(__builtin_bit_cast(double, b));
        return gbcast_bits<NP, 2 * O>(b | __builtin_bit_cast(unsigned long long, p));
    } else {
        return b;
    }
}

template <int NP, int L>
__device__ __forceinline__ C<L> gbcast_c(C<L> v, bool mine)
{
    C<L> r;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const unsigned long long br = mine ? __builtin_bit_cast(unsigned long long, v.re.v[l]) : 0ull;
        const unsigned long long bi = mine ? __builtin_bit_cast(unsigned long long, v.im.v[l]) : 0ull;
        r.re.v[l] = __builtin_bit_cast(double, gbcast_bits<NP>(br));
        r.im.v[l] = __builtin_bit_cast(double, gbcast_bits<NP>(bi));
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

// Everything a lane carries from one round to the next.  The path-level
// fields are identical in all lanes of a group; x, xp, xh are coordinate i.
// nh counts the accepted points before the current one that the predictor
// may use (x_p and, for orders above one, up to three older ones whose
// coordinates live in the history buffer and whose t values are tq).
template <int L>
struct Slot {
    int phase, sidx, n, succ, it, have_prev, pit, nh;
    int32_t steps, rejected, newton;
    int64_t gid;
    double t, tp, t1, h, dprev;
    double tq[3];
    C<L> x, xp, xh;
};

template <int L>
__device__ __forceinline__ void slot_init(Slot<L> &s)
{
    s.phase = PH_EMPTY;
    s.sidx = s.n = s.succ = s.it = s.have_prev = s.pit = s.nh = 0;
    s.steps = s.rejected = s.newton = 0;
    s.gid = 0;
    s.t = s.tp = s.t1 = s.h = s.dprev = 0.0;
    s.tq[0] = s.tq[1] = s.tq[2] = 0.0;
    s.x = s.xp = s.xh = c_zero<L>();
}

// Weights of the extrapolation predictor of order m (Section 2): the
// Lagrange basis of the nodes T[0..m] evaluated at t1, each a product of
// FP64 factors (t1 - T_i) / (T_j - T_i) in increasing i.
__device__ __forceinline__ void lagrange_weights(int m, const double *T, double t1, double *w)
{
    for (int j = 0; j <= m; ++j) {
        double wj = 1.0;
        for (int i = 0; i <= m; ++i) {
            if (i == j) continue;
            const double num = t1 - T[i];
            const double den = T[j] - T[i];
            wj = wj * (num / den);
        }
        w[j] = wj;
    }
}

// Run at most max_rounds rounds of the tracker on the slots of this wave, or
// until every slot is retired (the queue of the class is empty).  Returns
// true when the wave is retired.
template <int L, int NP, int KMAX, bool MIXED>
__device__ __forceinline__ bool run_rounds(const TrackArgs &a, const TrackClass &cl, Slot<L> &S, int max_rounds,
                           double *__restrict__ xsh, double *__restrict__ wsh)
{
    constexpr int LS = MIXED ? 1 : L;
    const int lane = threadIdx.x;
    const int g = lane / NP;
    const int i = lane % NP;
    const int base = g * NP;
    const ph_track_opts &o = a.o;
    const R<L> h3 = half_sqrt3_t<L>();
    // LDS views: xg = the group's current iterate, W(j, row) = entry of the
    // augmented matrix [J | -H] (column j = NP holds -H)
    double *xg = xsh + (size_t)g * NP * 2 * L;
    auto W = [&](int j, int row) -> double * {
        return wsh + (((size_t)g * (NP + 1) + j) * NP + row) * 2 * LS;
    };

    int phase = S.phase, sidx = S.sidx, n = S.n, succ = S.succ, it = S.it;
    int have_prev = S.have_prev, pit = S.pit, nh = S.nh;
    double tq0 = S.tq[0], tq1 = S.tq[1], tq2 = S.tq[2];
    const int order = o.predictor_order;
    // older history points of this lane's coordinate: [q][re,im][limb] rows
    // of the history buffer, one column per lane slot
    const int64_t hcol = (int64_t)blockIdx.x * 64 + lane;
    auto hist_get = [&](int q) -> C<L> {
        C<L> z;
#pragma unroll
        for (int l = 0; l < L; ++l) {
            z.re.v[l] = a.hist[((int64_t)(q * 2 + 0) * L + l) * a.hist_ld + hcol];
            z.im.v[l] = a.hist[((int64_t)(q * 2 + 1) * L + l) * a.hist_ld + hcol];
        }
        return z;
    };
    auto hist_put = [&](int q, const C<L> &z) {
#pragma unroll
        for (int l = 0; l < L; ++l) {
            a.hist[((int64_t)(q * 2 + 0) * L + l) * a.hist_ld + hcol] = z.re.v[l];
            a.hist[((int64_t)(q * 2 + 1) * L + l) * a.hist_ld + hcol] = z.im.v[l];
        }
    };
    int32_t steps = S.steps, rejected = S.rejected, newton = S.newton;
    int64_t gid = S.gid;
    double t = S.t, tp = S.tp, t1 = S.t1, h = S.h, dprev = S.dprev;
    C<L> x = S.x, xp = S.xp, xh = S.xh;

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
            atomicAdd(&a.stats[0], (unsigned long long)steps);
            atomicAdd(&a.stats[1], (unsigned long long)rejected);
            atomicAdd(&a.stats[2], (unsigned long long)newton);
            atomicAdd(&a.stats[3 + reason], 1ull);
        }
        phase = PH_EMPTY;
        n = 0;
    };

    bool retired = false;
    const long long t_start = a.budget ? wall_clock64() : 0;  // time-budgeted launches
    // what the evaluation reads of the slot's system, kept across rounds and
    // read again only when the slot moves to another system: the term-table
    // pointers, gamma, and this lane's equation and term range
    int k_sidx = -1, k_n = -1;
    const int4 *k_tdesc = nullptr;
    const double *k_coef = nullptr;
    const uint32_t *k_fac8 = nullptr;
    double k_gre = 0.0, k_gim = 0.0;
    int k_sub = NP, k_s0 = 0, k_s1 = 0;
    for (int round = 0; round < max_rounds; ++round) {
        // ---- refill: pop a path from the device queue of this class -------
        if (phase == PH_EMPTY) {
            unsigned long long id = 0;
            if (i == 0) id = atomicAdd(cl.queue, 1ull);
            id = __shfl(id, base);
            if ((int64_t)id >= cl.total) {
                phase = PH_RETIRED;
                n = 0;
            } else {
                const int64_t q = (int64_t)id;
                sidx = cl.sys_first;
                while (sidx + 1 < cl.sys_end && a.sys[sidx + 1].qoff <= q) ++sidx;
                const SysDesc &sd = a.sys[sidx];
                n = sd.n;
                const int64_t local = q - sd.qoff;
                gid = sd.path_off + local;
                const int64_t pid = sd.path_ids ? sd.path_ids[local] : local;
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
                succ = it = have_prev = pit = nh = 0;
                steps = rejected = newton = 0;
                phase = PH_STEP;
            }
        }
        const bool any_bad = gmax_d<NP>(c_bad<L>(x) ? 1.0 : 0.0) > 0.0;
        if (phase == PH_STEP && steps == 0) {
            if (o.h_min > o.h_init) finish(PH_R_STEP_UNDERFLOW);
            else if (any_bad) finish(PH_R_NAN);
        }
        // ---- stop when every slot of the wave is retired ------------------
        if (__all(phase == PH_RETIRED)) {
            retired = true;
            break;
        }

        // ---- predictor ----------------------------------------------------
        if (phase == PH_STEP) {
            if (steps >= o.max_steps) {
                finish(PH_R_MAX_STEPS);
            } else {
                ++steps;
                if (h > 1.0 - t) h = 1.0 - t;
                t1 = t + h;
                if (t1 >= 1.0 - 1e-15) t1 = 1.0;
                const int mo = nh < order ? nh : order;
                if (mo >= 2) {
                    // the current point and mo previous accepted points
                    const double T[5] = {t, tp, tq0, tq1, tq2};
                    double w[5];
                    lagrange_weights(mo, T, t1, w);
                    C<L> acc = c_add<L>(c_mul_d<L>(x, w[0]), c_mul_d<L>(xp, w[1]));
                    for (int j = 2; j <= mo; ++j) acc = c_add<L>(acc, c_mul_d<L>(hist_get(j - 2), w[j]));
                    xh = acc;
                } else if (have_prev) {
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
        if (busy && (sidx != k_sidx || n != k_n)) {
            const SysDesc &sd = a.sys[sidx];
            k_tdesc = sd.tdesc;
            k_coef = sd.coef;
            k_fac8 = sd.fac8;
            k_gre = sd.gre;
            k_gim = sd.gim;
            int sb4 = 4;
            while (sb4 < n) sb4 *= 2;
            // a helper's row holds 2L + kmax 2LS doubles of hand-over
            if (sb4 > NP || 2 * L + sd.kmax * 2 * LS > (NP + 1) * 2 * LS) sb4 = NP;
            k_sub = sb4;
            const int e = i % sb4;
            k_s0 = e < n ? sd.eq_off[e] : 0;
            k_s1 = e < n ? sd.eq_off[e + 1] : 0;
            k_sidx = sidx;
            k_n = n;
        }

        // ---- evaluate H and J at (xh, tt) ----------------------------------
        // sub = the smallest power of two >= n (at least 4); with nsh = NP / sub
        // lanes per equation, lane i = sr * sub + eq works on equation eq: the
        // nsh lanes of an equation take its terms round-robin (the term sweeps
        // run side by side) and lane eq adds every contribution in term order,
        // so the results do not depend on nsh.  A helper lane (sr > 0) hands its
        // term's value and partials over in its own row of the matrix, which
        // no equation uses (rows >= sub >= n), and clears the row afterwards.
#pragma unroll
        for (int l = 0; l < L; ++l) {
            xg[i * 2 * L + l] = xh.re.v[l];
            xg[i * 2 * L + L + l] = xh.im.v[l];
        }
#pragma unroll
        for (int j = 0; j <= NP; ++j) lds_put<LS>(W(j, i), c_zero<LS>());
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        const int sub = k_sub;
        const int nsh = NP / sub, eq = i % sub, sr = i / sub;
        // m-th double of row `row` of the group's matrix (hand-over slots)
        auto slot = [&](int row, int m) -> double * { return W(m / (2 * LS), row) + m % (2 * LS); };
        C<L> v = c_zero<L>();
        if (busy && eq < n) {
            double o1, oe;
            two_sum(1.0, -tt, o1, oe);
            R<L> omt = r_zero<L>();
            omt.v[0] = o1;
            if constexpr (L > 1) omt.v[1] = oe;
            const C<L> gs = c_mul_r<L>(c_from<L>(k_gre, k_gim), omt);
            auto X = [&](int var) -> C<L> {
                C<L> z;
#pragma unroll
                for (int l = 0; l < L; ++l) {
                    z.re.v[l] = xg[var * 2 * L + l];
                    z.im.v[l] = xg[var * 2 * L + L + l];
                }
                return z;
            };
            auto add_part = [&](uint32_t w, const C<LS> &part) {
                double *en = W(fac_var(w), eq);
                if constexpr (LS == 1) {
                    // FP64 entries: LDS atomic adds, which the lane issues
                    // without waiting for a read of the entry.  The lane is
                    // the only writer of its row and its LDS operations
                    // complete in order, so the sums are the same additions
                    // in the same order as a read, an add and a write.
                    __hip_atomic_fetch_add(en, part.re.v[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    __hip_atomic_fetch_add(en + 1, part.im.v[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                } else {
                    lds_put<LS>(en, c_add<LS>(lds_get<LS>(en), part));
                }
            };
            const int s0 = k_s0, s1 = k_s1;
            // a term's descriptor, coefficient and factor words (eight
            // slots per term, addressed by the term index alone) load
            // together; up to double double the lane reads its next term
            // while it sweeps the current one (quad double has no registers
            // to spare for that)
            constexpr bool AHEAD = L <= 2;
            auto fetch = [&](int s, int4 &d, C<L> &c, uint32_t (&fw)[KMAX]) {
                d = k_tdesc[s];
#pragma unroll
                for (int l = 0; l < L; ++l) {
                    c.re.v[l] = k_coef[(int64_t)s * 8 + l];
                    c.im.v[l] = k_coef[(int64_t)s * 8 + 4 + l];
                }
#pragma unroll
                for (int l = 0; l < KMAX; ++l) fw[l] = k_fac8[(int64_t)s * 8 + l];
            };
            int4 dn = {0, 0, 0, 0};
            C<L> cn = c_zero<L>();
            uint32_t fn[KMAX];
#pragma unroll
            for (int l = 0; l < KMAX; ++l) fn[l] = 0u;
            if (AHEAD && s0 + sr < s1) fetch(s0 + sr, dn, cn, fn);
            for (int sb = s0; sb < s1; sb += nsh) {
                const int s = sb + sr;
                int4 d = dn;
                C<L> c = cn;
                uint32_t fw[KMAX];
#pragma unroll
                for (int l = 0; l < KMAX; ++l) fw[l] = fn[l];
                if (AHEAD) {
                    if (s + nsh < s1) fetch(s + nsh, dn, cn, fn);
                } else if (s < s1) {
                    fetch(s, d, c, fw);
                }
                if (s < s1) {
                    c = d.z ? c_mul<L>(c, gs) : c_mul_d<L>(c, tt);
                    C<L> tv = c;
                    if (d.x > 0) {
                        tv = term_sweep<KMAX, true, (L <= 2)>(
                            d.x, fw, c, X, [&](int l, uint32_t w, const C<L> &part) {
                                const C<LS> pn = narrow<LS, L>(part);
                                if (sr == 0) {
                                    add_part(w, pn);
                                } else {
#pragma unroll
                                    for (int q = 0; q < LS; ++q) {
                                        *slot(i, 2 * L + l * 2 * LS + q) = pn.re.v[q];
                                        *slot(i, 2 * L + l * 2 * LS + LS + q) = pn.im.v[q];
                                    }
                                }
                            });
                    }
                    if (sr == 0) {
                        v = c_add<L>(v, tv);
                    } else {
#pragma unroll
                        for (int q = 0; q < L; ++q) {
                            *slot(i, q) = tv.re.v[q];
                            *slot(i, L + q) = tv.im.v[q];
                        }
                    }
                }
                if (nsh > 1) {
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                    if (sr == 0) {
                        // the helpers' terms, in term order, partials in the
                        // order the sweep issues them (last factor first)
                        for (int q = 1; q < nsh && sb + q < s1; ++q) {
                            const int hrow = i + q * sub;
                            const int4 d = k_tdesc[sb + q];
                            for (int l = d.x - 1; l >= 0; --l) {
                                C<LS> pn;
#pragma unroll
                                for (int z = 0; z < LS; ++z) {
                                    pn.re.v[z] = *slot(hrow, 2 * L + l * 2 * LS + z);
                                    pn.im.v[z] = *slot(hrow, 2 * L + l * 2 * LS + LS + z);
                                }
                                add_part(k_fac8[(int64_t)(sb + q) * 8 + l], pn);
                            }
                            C<L> tv;
#pragma unroll
                            for (int z = 0; z < L; ++z) {
                                tv.re.v[z] = *slot(hrow, z);
                                tv.im.v[z] = *slot(hrow, L + z);
                            }
                            v = c_add<L>(v, tv);
                        }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                }
            }
            if (sr == 0) lds_put<LS>(W(NP, i), narrow<LS, L>(c_sub<L>(c_zero<L>(), v)));
        }
        if (nsh > 1 && sr > 0) {
#pragma unroll
            for (int j = 0; j <= NP; ++j) lds_put<LS>(W(j, i), c_zero<LS>());
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");

        // ---- correct: MGS least squares on [J | -H], row i in lane i ------
        // residual at the point where the Newton system is formed (the
        // convergence test compares it with ||J||_F, Section 2)
        const double hres = gmax_d<NP>((busy && i < n) ? c_absd<LS>(lds_get<LS>(W(NP, i))) : 0.0);
        double fro = 0.0;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            C<LS> w = lds_get<LS>(W(j, i));
            fro += w.re.v[0] * w.re.v[0] + w.im.v[0] * w.im.v[0];
        }
        fro = sqrt(gsum_d<NP>(fro));
        bool sing = false;
        C<LS> acc = c_zero<LS>();  // r_{i,rhs}, then the back-substitution value
        // the column loops address LDS only, so they stay rolled (code size)
#pragma unroll 1
        for (int k = 0; k < n; ++k) {
            {  // group-uniform
                C<LS> wk = lds_get<LS>(W(k, i));
                R<LS> nr = gsum_r<NP, LS>(c_abs2<LS>(wk));
                R<LS> rkk, inv;
                if constexpr (LS == 1) {
                    // FP64: the norm and its reciprocal from one reciprocal
                    // square root refined by two coupled Newton steps
                    // (Goldschmidt: g -> sqrt(x), h -> 1 / (2 sqrt(x))), in
                    // place of a square root and a division in series
                    const double x = nr.v[0];
                    const double y = __builtin_amdgcn_rsq(x);
                    double g = x * y, h = 0.5 * y;
#pragma unroll
                    for (int it = 0; it < 2; ++it) {
                        const double r = __builtin_fma(-g, h, 0.5);
                        g = __builtin_fma(g, r, g);
                        h = __builtin_fma(h, r, h);
                    }
                    // a norm below the normal range, zero or NaN counts as zero
                    // (singular), infinity stays NaN (singular as well)
                    rkk.v[0] = x >= 0x1p-1022 ? g : 0.0;
                    inv.v[0] = 2.0 * h;
                } else {
                    rkk = r_sqrt<LS>(nr);
                }
                if (!(rkk.v[0] > a.eps_sing * fro)) sing = true;
                if (sing) break;
                {
                    if constexpr (LS != 1) inv = r_div<LS>(r_from<LS>(1.0), rkk);
                    C<LS> q = c_mul_r<LS>(wk, inv);
                    // projection of column j on q: r = q^H w_j (group sum),
                    // w_j -= r q; column k is dead after step k, so R(k, j)
                    // goes to row j of it
                    auto proj = [&](int j) -> C<LS> {
                        double *ej = W(j, i);
                        C<LS> wj = lds_get<LS>(ej);
                        C<LS> r = gsum_c<NP, LS>(c_cmul<LS>(q, wj));
                        lds_put<LS>(ej, c_sub<LS>(wj, c_mul<LS>(r, q)));
                        return r;
                    };
                    if constexpr (LS == 1) {
                        // FP64 solves are latency bound: four columns at a
                        // time, so their group sums interleave; the stores
                        // of R(k, j) follow, one per lane
                        int j = k + 1;
#pragma unroll 1
                        for (; j + 3 < n; j += 4) {
                            const C<LS> r0 = proj(j), r1 = proj(j + 1), r2 = proj(j + 2), r3 = proj(j + 3);
                            const int d = i - j;
                            if (d >= 0 && d < 4)
                                lds_put<LS>(W(k, i), d == 0 ? r0 : (d == 1 ? r1 : (d == 2 ? r2 : r3)));
                        }
#pragma unroll 1
                        for (; j < n; ++j) {
                            const C<LS> r = proj(j);
                            if (i == j) lds_put<LS>(W(k, j), r);
                        }
                        const C<LS> r = proj(NP);
                        if (i == k) acc = r;
                    } else {
#pragma unroll 1
                        for (int j = k + 1; j <= NP; ++j) {
                            if (j == n && j < NP) j = NP;  // skip the padding columns
                            const C<LS> r = proj(j);
                            if (i == k && j == NP) acc = r;
                            if (j < NP && i == j) lds_put<LS>(W(k, j), r);
                        }
                    }
                    if (i == k) lds_put<LS>(W(k, k), C<LS>{rkk, r_zero<LS>()});
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        // back substitution R dx = r_rhs, column oriented: lane i keeps acc_i;
        // every lane forms 1 / R(i, i) first, side by side, so that no
        // division sits on the serial chain of the substitution
        C<LS> dxi = c_zero<LS>();
        R<LS> inv_i = r_zero<LS>();
        if (!sing && i < n) inv_i = r_div<LS>(r_from<LS>(1.0), lds_get<LS>(W(i, i)).re);
#pragma unroll 1
        for (int k = n - 1; k >= 0; --k) {
            if (!sing) {
                C<LS> dk = c_zero<LS>();
                if (i == k) {
                    dk = c_mul_r<LS>(acc, inv_i);
                    dxi = dk;
                }
                if constexpr (NP <= 16)
                    dk = gbcast_c<NP, LS>(dk, i == k);
                else
                    dk = shfl_c<LS>(dk, base + k);
                if (i < k) {
                    C<LS> rik = lds_get<LS>(W(i, k));  // R(i, k), stored in column i, row k
                    acc = c_sub<LS>(acc, c_mul<LS>(rik, dk));
                }
            }
        }
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
                const double sx = xn > 1.0 ? xn : 1.0;
                if (dn != dn || xn != xn) {
                    reject = true;
                } else if (dn <= o.tol_dx * sx && hres <= o.tol_res * fro * sx) {
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
                if (order >= 2) {
                    // shift the history: older points move down, x_p joins
                    if (nh >= 3) hist_put(2, hist_get(1));
                    if (nh >= 2) hist_put(1, hist_get(0));
                    hist_put(0, xp);
                    tq2 = tq1;
                    tq1 = tq0;
                    tq0 = tp;
                }
                tp = t;
                xp = x;
                have_prev = 1;
                if (nh < 4) ++nh;
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
            // halving, or polish_max steps were taken; an update that is not
            // finite ends the polish without being applied
            bool done = false;
            if (sing) {
                done = true;
            } else {
                const double dn = gmax_d<NP>(i < n ? c_absd<LS>(dxi) : 0.0);
                if (!isfinite(dn) || (pit > 0 && !(dn < 0.5 * dprev))) {
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
            if (done) {
                // the endpoint must be finite and within diverge_norm
                const bool bad = gmax_d<NP>((i < n && c_bad<L>(x)) ? 1.0 : 0.0) > 0.0;
                const double xe = gmax_d<NP>(i < n ? c_absd<L>(x) : 0.0);
                finish(bad ? PH_R_NAN : (xe > o.diverge_norm ? PH_R_DIVERGED : PH_R_SUCCESS));
            }
        }
        // round schedule with a time budget: every wave of the launch stops
        // after the round in which the budget ran out (wave-uniform clock),
        // so waves with cheap rounds do not wait for the others at the end
        // of a launch of a fixed round count
        if (a.budget && (unsigned long long)(wall_clock64() - t_start) >= a.budget) break;
    }
    S.phase = phase;
    S.sidx = sidx;
    S.n = n;
    S.succ = succ;
    S.it = it;
    S.have_prev = have_prev;
    S.pit = pit;
    S.nh = nh;
    S.tq[0] = tq0;
    S.tq[1] = tq1;
    S.tq[2] = tq2;
    S.steps = steps;
    S.rejected = rejected;
    S.newton = newton;
    S.gid = gid;
    S.t = t;
    S.tp = tp;
    S.t1 = t1;
    S.h = h;
    S.dprev = dprev;
    S.x = x;
    S.xp = xp;
    S.xh = xh;
    return retired;
}

// LDS of one wave for lane count NP: the iterate (64 lanes x 2L doubles) and
// the augmented matrices (64/NP paths x (NP+1) columns x NP rows x 2LS).
template <int L, int NP, bool MIXED>
__host__ __device__ constexpr size_t track_lds_doubles()
{
    return 64 * 2 * L + (size_t)(64 / NP) * (NP + 1) * NP * 2 * (MIXED ? 1 : L);
}

// Dispatch a block to its lane-count class.  Classes with lane counts 4, 8,
// 16, 32 own consecutive block ranges; each runs its own work queue.
// NPSEL > 0: the largest class present, so smaller launches do not carry the
// code (and the registers) of the n <= 32 class; NPSEL < 0: the launch has
// the single class -NPSEL and carries only its code (a single homotopy).
template <int L, int KMAX, bool MIXED, int NPSEL>
__device__ __forceinline__ bool run_class(const TrackArgs &a, Slot<L> &S, int max_rounds, double *lds)
{
    const int b = blockIdx.x;
    int c = 0;
    while (c < 3 && b >= a.cls[c].block_end) ++c;
    const TrackClass &cl = a.cls[c];
    double *xsh = lds;
    double *wsh = lds + 64 * 2 * L;
    if constexpr (NPSEL < 0) {
        return run_rounds<L, -NPSEL, KMAX, MIXED>(a, cl, S, max_rounds, xsh, wsh);
    } else {
    constexpr int NPMAX = NPSEL;
    if (cl.np == 4) return run_rounds<L, 4, KMAX, MIXED>(a, cl, S, max_rounds, xsh, wsh);
    if (cl.np == 8 || NPMAX == 8) return run_rounds<L, 8, KMAX, MIXED>(a, cl, S, max_rounds, xsh, wsh);
    if constexpr (NPMAX >= 16)
        if (cl.np == 16 || NPMAX == 16) return run_rounds<L, 16, KMAX, MIXED>(a, cl, S, max_rounds, xsh, wsh);
    if constexpr (NPMAX >= 32) return run_rounds<L, 32, KMAX, MIXED>(a, cl, S, max_rounds, xsh, wsh);
    return true;
    }
}

// One kernel for both schedules.  Persistent (a.state == NULL): every wave
// runs until its class queue is empty.  Rounds (a.state != NULL): every
// launch runs a.rounds rounds and keeps each lane's slot in device memory
// between launches; the host replays a captured graph of {clear counter,
// this kernel} and reads the number of waves still active.
// Two waves per SIMD: the double-double and quad-double state machines want
// more than 256 registers; the compiler keeps them within 256 by spilling
// a few values to scratch, which costs far less than running one wave per
// SIMD (measured: 1.6x on the many-system double-double batch, 1.3x on the
// 65536-path quad-double workload).
template <int L, int KMAX, bool MIXED, int NPSEL>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) track_kernel(TrackArgs a)
{
    extern __shared__ double lds[];
    Slot<L> *st = a.state ? reinterpret_cast<Slot<L> *>(a.state) + (size_t)blockIdx.x * 64 + threadIdx.x
                          : nullptr;
    Slot<L> S;
    if (st)
        S = *st;
    else
        slot_init<L>(S);
    if (__all(S.phase == PH_RETIRED)) return;
    const bool retired = run_class<L, KMAX, MIXED, NPSEL>(a, S, st ? a.rounds : 0x7fffffff, lds);
    if (st) {
        *st = S;
        if (!retired && threadIdx.x == 0) atomicAdd(a.active, 1u);
    }
}

template <int L>
__global__ void __launch_bounds__(256) slot_init_kernel(void *state, int64_t nslots)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nslots) return;
    Slot<L> S;
    slot_init<L>(S);
    reinterpret_cast<Slot<L> *>(state)[k] = S;
}


}  // namespace ph
