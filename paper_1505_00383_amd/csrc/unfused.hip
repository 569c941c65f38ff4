// unfused.hip -- the paper's three-kernel evaluation (Section 3, Tables 4-6
// and 8), kept as a measured ablation of the fused kernels:
//
//   coeff: c_tau(t_p) = t_p c_tau (target term) or gamma (1 - t_p) c_tau (start
//          term) for every (term, point), written to device memory;
//   mon:   per (term, point) the value c x^a and the k partial derivatives
//          (reverse-mode products of Table 6, exponents applied), written to
//          one slot each ("vertical" layout: slot-major, point fastest);
//   sum:   per (output entry, point) the sum of its slots: H_i over the
//          values of equation i's terms, J_ij over the partials by x_j.
//
// Every array is structure-of-arrays with the point index fastest, as in the
// rest of the library.  The intermediate arrays (coefficients and slots)
// live in a buffer of the term table that ph_eval_prepare sizes; points
// beyond its capacity run in several chunks.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ph_arith.hpp"
#include "ph_internal.hpp"
#include "ph_sweep.hpp"

namespace ph {

struct UArgs {
    const int32_t *eq_off;
    const int4 *tdesc;
    const uint32_t *fac;
    const double *coef;
    const int32_t *u_slot, *u_off, *u_list;
    const double *t, *x;
    double *val, *jac;
    double *cff;   // [term][re,im][limb][lu]
    double *mon;   // [slot][re,im][limb][lu]
    int64_t npts, ld, lu;
    int64_t n_terms, n_entries;
    double gre, gim;
    int n_eq, n_var;
};

template <int L>
__device__ __forceinline__ void put_c(double *base, int64_t row, int64_t ld, int64_t p, const C<L> &z)
{
#pragma unroll
    for (int l = 0; l < L; ++l) {
        base[((row * 2 + 0) * L + l) * ld + p] = z.re.v[l];
        base[((row * 2 + 1) * L + l) * ld + p] = z.im.v[l];
    }
}

template <int L>
__device__ __forceinline__ C<L> get_c(const double *base, int64_t row, int64_t ld, int64_t p)
{
    C<L> z;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        z.re.v[l] = base[((row * 2 + 0) * L + l) * ld + p];
        z.im.v[l] = base[((row * 2 + 1) * L + l) * ld + p];
    }
    return z;
}

// coeff: one lane per point, the waves of a block stride over the terms of
// their block's term range.
template <int L>
__global__ void __launch_bounds__(256) coeff_kernel(UArgs a)
{
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t p = (int64_t)blockIdx.x * 64 + lane;
    if (p >= a.npts) return;
    const double tv = a.t ? a.t[p] : 1.0;
    double o1, oe;
    two_sum(1.0, -tv, o1, oe);
    R<L> omt = r_zero<L>();
    omt.v[0] = o1;
    if constexpr (L > 1) omt.v[1] = oe;
    const C<L> gs = a.t ? c_mul_r<L>(c_from<L>(a.gre, a.gim), omt) : c_zero<L>();
    const int64_t per = (a.n_terms + gridDim.y - 1) / gridDim.y;
    const int64_t s0 = blockIdx.y * per, s1 = s0 + per < a.n_terms ? s0 + per : a.n_terms;
    for (int64_t s = s0 + w; s < s1; s += blockDim.x >> 6) {
        C<L> c;
#pragma unroll
        for (int l = 0; l < L; ++l) {
            c.re.v[l] = a.coef[s * 8 + l];
            c.im.v[l] = a.coef[s * 8 + 4 + l];
        }
        c = a.tdesc[s].z ? c_mul<L>(c, gs) : c_mul_d<L>(c, tv);
        put_c<L>(a.cff, s, a.lu, p, c);
    }
}

// mon: the block's 64 points staged in LDS, one wave per term.
template <int L, int KMAX>
__global__ void __launch_bounds__(256) mon_kernel(UArgs a)
{
    extern __shared__ double xl[];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int W = blockDim.x >> 6;
    const int64_t p = (int64_t)blockIdx.x * 64 + lane;
    const bool act = p < a.npts;
    for (int r = w; r < a.n_var * 2 * L; r += W) xl[r * 64 + lane] = act ? a.x[(int64_t)r * a.ld + p] : 0.0;
    __syncthreads();
    if (!act) return;
    auto X = [&](int var) -> C<L> {
        C<L> z;
#pragma unroll
        for (int l = 0; l < L; ++l) {
            z.re.v[l] = xl[((var * 2 + 0) * L + l) * 64 + lane];
            z.im.v[l] = xl[((var * 2 + 1) * L + l) * 64 + lane];
        }
        return z;
    };
    const int64_t per = (a.n_terms + gridDim.y - 1) / gridDim.y;
    const int64_t s0 = blockIdx.y * per, s1 = s0 + per < a.n_terms ? s0 + per : a.n_terms;
    for (int64_t s = s0 + w; s < s1; s += W) {
        const int4 d = a.tdesc[s];
        const int64_t slot = a.u_slot[s];
        const C<L> c = get_c<L>(a.cff, s, a.lu, p);
        if (d.x == 0) {
            put_c<L>(a.mon, slot, a.lu, p, c);
            continue;
        }
        uint32_t fw[KMAX];
#pragma unroll
        for (int l = 0; l < KMAX; ++l)
            if (l < d.x) fw[l] = a.fac[d.y + l];
        const C<L> v = term_sweep<KMAX, true, (L == 1)>(
            d.x, fw, c, X, [&](int l, uint32_t, const C<L> &part) { put_c<L>(a.mon, slot + 1 + l, a.lu, p, part); });
        put_c<L>(a.mon, slot, a.lu, p, v);
    }
}

// sum: one wave per output entry (wave-uniform slot list), lane per point.
template <int L>
__global__ void __launch_bounds__(256) sum_kernel(UArgs a)
{
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t p = (int64_t)blockIdx.x * 64 + lane;
    if (p >= a.npts) return;
    const int64_t per = (a.n_entries + gridDim.y - 1) / gridDim.y;
    const int64_t e0 = blockIdx.y * per, e1 = e0 + per < a.n_entries ? e0 + per : a.n_entries;
    for (int64_t e = e0 + w; e < e1; e += blockDim.x >> 6) {
        C<L> acc = c_zero<L>();
        for (int q = a.u_off[e]; q < a.u_off[e + 1]; ++q) acc = c_add<L>(acc, get_c<L>(a.mon, a.u_list[q], a.lu, p));
        if (e < a.n_eq)
            put_c<L>(a.val, e, a.ld, p, acc);
        else if (a.jac)
            put_c<L>(a.jac, e - a.n_eq, a.ld, p, acc);
    }
}

template <int L>
static int unfused_run(const DevTable &tab, const UArgs &a0, hipStream_t st)
{
    UArgs a = a0;
    const unsigned bx = (unsigned)((a.npts + 63) / 64);
    // enough blocks to fill the chip; each block's waves stride over a range
    auto gy = [&](int64_t items) {
        int64_t g = 1;
        while ((int64_t)bx * g < 2048 && g * 4 < items) g *= 2;
        return (unsigned)g;
    };
    hipLaunchKernelGGL(coeff_kernel<L>, dim3(bx, gy(a.n_terms)), dim3(256), 0, st, a);
    const size_t lds = (size_t)a.n_var * 2 * L * 64 * sizeof(double);
    if (tab.kmax <= 8)
        hipLaunchKernelGGL((mon_kernel<L, 8>), dim3(bx, gy(a.n_terms)), dim3(256), lds, st, a);
    else if (tab.kmax <= 16)
        hipLaunchKernelGGL((mon_kernel<L, 16>), dim3(bx, gy(a.n_terms)), dim3(256), lds, st, a);
    else
        hipLaunchKernelGGL((mon_kernel<L, 32>), dim3(bx, gy(a.n_terms)), dim3(256), lds, st, a);
    hipLaunchKernelGGL(sum_kernel<L>, dim3(bx, gy(a.n_entries)), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "unfused kernels launch");
    return PH_OK;
}

int unfused_launch(const DevTable &tab, const double gamma[2], int prec, int64_t npts,
                   const double *t, const double *x, int64_t ld, double *val, double *jac,
                   hipStream_t st)
{
    if ((size_t)tab.n_var * 2 * prec * 64 * sizeof(double) > 160 * 1024)
        return fail(PH_EUNSUPPORTED, "unfused evaluation stages the points in LDS (n * prec <= 160)");
    // the intermediate arrays were sized by ph_eval_prepare: the points run in
    // chunks of the capacity they hold at this precision
    const size_t per_point = (size_t)(tab.n_terms + tab.u_slots) * 2 * prec * sizeof(double);
    const int64_t cap = tab.u_scratch ? (int64_t)(tab.u_scratch_bytes / per_point) / 64 * 64 : 0;
    if (cap < 64)
        return fail(PH_EINVAL, "unfused evaluation: size its arrays with ph_eval_prepare (unfused_points > 0)");
    UArgs a;
    a.eq_off = tab.eq_off;
    a.tdesc = tab.tdesc;
    a.fac = tab.fac;
    a.coef = tab.coef;
    a.u_slot = tab.u_slot;
    a.u_off = tab.u_off;
    a.u_list = tab.u_list;
    a.ld = ld;
    a.n_terms = tab.n_terms;
    a.n_entries = (int64_t)tab.n_eq * (1 + tab.n_var);
    a.gre = gamma ? gamma[0] : 1.0;
    a.gim = gamma ? gamma[1] : 0.0;
    a.n_eq = tab.n_eq;
    a.n_var = tab.n_var;
    for (int64_t p0 = 0; p0 < npts; p0 += cap) {
        const int64_t m = npts - p0 < cap ? npts - p0 : cap;
        a.npts = m;
        a.lu = (m + 63) / 64 * 64;
        a.cff = static_cast<double *>(tab.u_scratch);
        a.mon = a.cff + (size_t)tab.n_terms * 2 * prec * a.lu;
        a.t = t ? t + p0 : nullptr;
        a.x = x + p0;
        a.val = val + p0;
        a.jac = jac ? jac + p0 : nullptr;
        int rc;
        switch (prec) {
        case 1: rc = unfused_run<1>(tab, a, st); break;
        case 2: rc = unfused_run<2>(tab, a, st); break;
        default: rc = unfused_run<4>(tab, a, st); break;
        }
        if (rc) return rc;
    }
    return PH_OK;
}

}  // namespace ph
