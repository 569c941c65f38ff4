// eval_dd.hip -- double-double values and Jacobian of gamma (1-t) g + t f
// (Eq. (1)) with the Jacobian row of the equation in flight held on chip, for
// systems with n <= 32 unknowns, terms of at most 8 factors and exponents
// whose powers x^(a-1) fit the LDS power table (the fast-path records).
//
// The row of one equation is 32 columns of complex double doubles, 128
// doubles per point: more than a lane can keep beside its working registers
// in the architectural register file.  It lives in the 256 accumulation
// registers (AGPRs) instead, column j in a[8j .. 8j+7] = {re hi, re lo, im hi,
// im lo} (two dwords each), and the kernel runs one wave per SIMD so that each
// wave owns 256 architectural registers for the term sweep and 256 AGPRs for
// the row.  A partial derivative is added to its column (a wave-uniform
// index) by reading the eight dwords with the GPR indexing mode applied to
// v_accvgpr_read, one TwoProd / TwoSum / FastTwoSum update per component in
// ordinary registers, and eight indexed v_accvgpr_write.  H and J leave the
// kernel once per equation (compulsory bytes only).
//
// Everything else follows the complex-double fast path: one lane = one point,
// the workgroup's waves share 64 points whose x and x^2 (x^3 when exponents
// reach 4) are staged in LDS in the double-double layout
// ((plane * n + v) * 4 + {re hi, re lo, im hi, im lo}) * 64 + lane, each wave
// takes whole equations, and terms come as 256-byte records through scalar
// loads, grouped by (factors, factors with a >= 2), the next record fetched
// one term ahead.  Per term (Section 1 decomposition, Table 6 products):
// coefficient times t or gamma (1 - t), times the powers (balanced tree),
// the suffix products, then one forward pass issuing each partial beside the
// next prefix product: 3k - 3 + #{a >= 2} complex products.
#include <hip/hip_runtime.h>

#include "ph_arith.hpp"
#include "ph_arow.hpp"
#include "ph_internal.hpp"

namespace ph {

struct DDArgs {
    const double *t;
    const double *x;
    double *val;
    double *jac;
    int64_t npts, ld;
    double gre, gim;
    int n_eq, n_var, eq_stride, planes;
};

// hi + lo += e * (ph + pl): TwoProd of e and the leading limb, TwoSum with
// the leading limb of the sum, every lower-order term folded into the error
// and one FastTwoSum (the double-word addition without a second TwoSum: its
// error is a few u^2 times |hi + lo| + |e (ph + pl)|, which is what the
// evaluation's accuracy is stated against).  e is a small integer exponent.
__device__ __forceinline__ void dd_axpy(double &hi, double &lo, double e, double ph, double pl)
{
    double p, pe, s, se;
    two_prod(e, ph, p, pe);
    two_sum(hi, p, s, se);
    se += lo + __builtin_fma(e, pl, pe);
    fast_two_sum(s, se, hi, lo);
}

// hi + lo += ph + pl, the same without the scaling.
__device__ __forceinline__ void dd_acc(double &hi, double &lo, double ph, double pl)
{
    double s, se;
    two_sum(hi, ph, s, se);
    se += lo + pl;
    fast_two_sum(s, se, hi, lo);
}

__device__ __forceinline__ void row_axpy(ARow &row, uint32_t jo, double e, const C<2> &d)
{
    double rh, rl, ih, il;
    row.read(jo, rh, rl, ih, il);
    dd_axpy(rh, rl, e, d.re.v[0], d.re.v[1]);
    dd_axpy(ih, il, e, d.im.v[0], d.im.v[1]);
    row.write(jo, rh, rl, ih, il);
}

__device__ __forceinline__ void val_acc(C<2> &v, const C<2> &d)
{
    dd_acc(v.re.v[0], v.re.v[1], d.re.v[0], d.re.v[1]);
    dd_acc(v.im.v[0], v.im.v[1], d.im.v[0], d.im.v[1]);
}

// a double-double complex from the LDS staging rows at byte offset off
__device__ __forceinline__ C<2> lds2(const char *__restrict__ xb, uint32_t off, int lane)
{
    const double *p = reinterpret_cast<const double *>(xb + off);
    C<2> z;
    z.re.v[0] = p[lane];
    z.re.v[1] = p[64 + lane];
    z.im.v[0] = p[128 + lane];
    z.im.v[1] = p[192 + lane];
    return z;
}

// One term with K factors, the first M of them with a >= 2 (same product
// order as the complex-double fast path).
template <int K, int M>
__device__ __forceinline__ void mfast_sweep(const MHead<2> &h, const MTerm *__restrict__ rnext, MHead<2> &hnext,
                                            const char *__restrict__ xb, int lane, C<2> cf, ARow &row,
                                            C<2> &v)
{
    C<2> xv[K], pw[M > 0 ? M : 1], sf[K];
#pragma unroll
    for (int l = 0; l < K; ++l) xv[l] = lds2(xb, h.xo[l], lane);
#pragma unroll
    for (int l = 0; l < M; ++l) pw[l] = lds2(xb, h.po[l], lane);
    hnext = mfast_head<K, M, 2>(rnext);
    if constexpr (M > 0) {
#pragma unroll
        for (int st = 1; st < M; st *= 2) {
#pragma unroll
            for (int l = 0; l + st < M; l += 2 * st) pw[l] = c_mul<2>(pw[l], pw[l + st]);
        }
        cf = c_mul<2>(cf, pw[0]);
    }
    sf[K - 1] = xv[K - 1];
#pragma unroll
    for (int l = K - 2; l >= 1; --l) sf[l] = c_mul<2>(sf[l + 1], xv[l]);
    C<2> q = cf;
#pragma unroll
    for (int l = 0; l < K - 1; ++l) {
        const C<2> part = c_mul<2>(q, sf[l + 1]);
        q = c_mul<2>(q, xv[l]);
        row_axpy(row, h.jo[l], h.a[l], part);
    }
    val_acc(v, c_mul<2>(q, xv[K - 1]));
    row_axpy(row, h.jo[K - 1], h.a[K - 1], q);
}

__device__ __forceinline__ C<2> mcoef(const MHead<2> &h, const C<2> &gs, double tv)
{
    C<2> c;
    c.re.v[0] = h.c[0];
    c.re.v[1] = h.c[1];
    c.im.v[0] = h.c[2];
    c.im.v[1] = h.c[3];
    return (h.sel & 1) ? c_mul<2>(c, gs) : c_mul_d<2>(c, tv);
}

template <int K, int M, int KF>
__device__ __forceinline__ void mfast_groups(const int32_t *__restrict__ run, const MTerm *__restrict__ mt,
                                             const char *__restrict__ xb, int lane, const C<2> &gs,
                                             double tv, ARow &row, C<2> &v)
{
    constexpr int g = drun_group(K, M);
    const int s0 = run[g], s1 = run[g + 1];
    if (s0 < s1) {
        MHead<2> h = mfast_head<K, M, 2>(mt + s0);
        for (int s = s0; s < s1; ++s) {
            const MTerm *rn = mt + (s + 1 < s1 ? s + 1 : s);
            MHead<2> hn;
            mfast_sweep<K, M>(h, rn, hn, xb, lane, mcoef(h, gs, tv), row, v);
            h = hn;
        }
    }
    if constexpr (M < K)
        mfast_groups<K, M + 1, KF>(run, mt, xb, lane, gs, tv, row, v);
    else if constexpr (K < KF)
        mfast_groups<K + 1, 0, KF>(run, mt, xb, lane, gs, tv, row, v);
}

__device__ __forceinline__ void st_nt(double *p, double v) { __builtin_nontemporal_store(v, p); }

// One wave per SIMD: 256 architectural registers for the sweep, 256 AGPRs
// for the row (at most four waves per workgroup).
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
eval_dd_arow_kernel(DDArgs a, const int32_t *__restrict__ d_run, const MTerm *__restrict__ mterm,
                    const int32_t *__restrict__ d_deg)
{
    extern __shared__ double xl[];
    const char *xb = reinterpret_cast<const char *>(xl);
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int W = blockDim.x >> 6;
    const int64_t p = (int64_t)blockIdx.x * 64 + lane;
    const bool act = p < a.npts;
    const int nv = a.n_var;
    // stage x and its powers: plane q holds x^(q+1), rows {re hi, re lo, im hi, im lo}
    for (int var = w; var < nv; var += W) {
        C<2> x1 = c_zero<2>();
        if (act) {
#pragma unroll
            for (int l = 0; l < 2; ++l) {
                x1.re.v[l] = a.x[(int64_t)(var * 4 + l) * a.ld + p];
                x1.im.v[l] = a.x[(int64_t)(var * 4 + 2 + l) * a.ld + p];
            }
        }
        C<2> z = x1;
        for (int q = 0; q < a.planes; ++q) {
            double *row = xl + (size_t)((q * nv + var) * 4) * 64;
            row[lane] = z.re.v[0];
            row[64 + lane] = z.re.v[1];
            row[128 + lane] = z.im.v[0];
            row[192 + lane] = z.im.v[1];
            z = c_mul<2>(z, x1);
        }
    }
    if (w == 0) {
        double *row = xl + (size_t)(a.planes * nv * 4) * 64;
        row[lane] = 1.0;
        row[64 + lane] = 0.0;
        row[128 + lane] = 0.0;
        row[192 + lane] = 0.0;
    }
    __syncthreads();

    // c(t): t for target terms, gamma (1 - t) for start terms, (1 - t) exact
    // in two limbs
    double tv = 1.0;
    if (a.t) tv = act ? a.t[p] : 0.0;
    C<2> gs = c_zero<2>();
    if (a.t) {
        double o, oe;
        two_sum(1.0, -tv, o, oe);
        R<2> omt;
        omt.v[0] = o;
        omt.v[1] = oe;
        gs = c_mul_r<2>(c_from<2>(a.gre, a.gim), omt);
    }

    for (int i = blockIdx.y * W + w; i < a.n_eq; i += a.eq_stride) {
        ARow row;
        row.zero();
        C<2> v = c_zero<2>();
        const int32_t *run = d_run + i * DRUN;
        for (int s = run[0]; s < run[1]; ++s) {
            MHead<2> h = mfast_head<0, 0, 2>(mterm + s);
            val_acc(v, mcoef(h, gs, tv));
        }
        mfast_groups<1, 0, 8>(run, mterm, xb, lane, gs, tv, row, v);
        // total-degree start part: gamma (1-t) (x_i^d - 1), derivative d x_i^(d-1)
        const int d = d_deg[i];
        if (d > 0 && a.t) {
            const C<2> xi = lds2(xb, (uint32_t)(i * 4 * 64 * 8), lane);
            C<2> pw = c_from<2>(1.0, 0.0), base = xi;  // pw = x_i^(d-1)
            for (int e = d - 1; e > 0; e >>= 1) {
                if (e & 1) pw = c_mul<2>(pw, base);
                if (e > 1) base = c_mul<2>(base, base);
            }
            const C<2> gp = c_mul<2>(gs, pw);
            val_acc(v, c_sub<2>(c_mul<2>(gp, xi), gs));
            row_axpy(row, (uint32_t)(8 * i), (double)d, gp);
        }
        if (act) {
            double *hv = a.val + (int64_t)(i * 4) * a.ld + p;
            st_nt(hv, v.re.v[0]);
            st_nt(hv + a.ld, v.re.v[1]);
            st_nt(hv + 2 * a.ld, v.im.v[0]);
            st_nt(hv + 3 * a.ld, v.im.v[1]);
            double *jr = a.jac + (int64_t)i * nv * 4 * a.ld + p;
            for (int j = 0; j < nv; ++j) {
                double rh, rl, ih, il;
                row.read((uint32_t)(8 * j), rh, rl, ih, il);
                double *q = jr + (int64_t)(j * 4) * a.ld;
                st_nt(q, rh);
                st_nt(q + a.ld, rl);
                st_nt(q + 2 * a.ld, ih);
                st_nt(q + 3 * a.ld, il);
            }
        }
    }
}

int dd_fast_launch(const DevTable &tab, const double gamma[2], int64_t npts, const double *t,
                   const double *x, int64_t ld, double *val, double *jac, int W, int G,
                   hipStream_t st)
{
    DDArgs a;
    a.t = t;
    a.x = x;
    a.val = val;
    a.jac = jac;
    a.npts = npts;
    a.ld = ld;
    a.gre = gamma ? gamma[0] : 1.0;
    a.gim = gamma ? gamma[1] : 0.0;
    a.n_eq = tab.n_eq;
    a.n_var = tab.n_var;
    a.planes = tab.dfast_planes;
    W = W < 1 ? 1 : (W > 4 ? 4 : W);
    if (W > tab.n_eq) W = tab.n_eq;
    if (G < 1) G = 1;
    while (G > 1 && G * W > tab.n_eq) G >>= 1;
    a.eq_stride = G * W;
    const size_t lds = ((size_t)tab.dfast_planes * tab.n_var * 4 + 4) * 64 * sizeof(double);
    dim3 grid((unsigned)((npts + 63) / 64), (unsigned)G);
    hipLaunchKernelGGL(eval_dd_arow_kernel, grid, dim3(64 * W), lds, st, a, tab.d_run, tab.mterm, tab.d_deg);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "eval_dd_arow_kernel launch");
    return PH_OK;
}

}  // namespace ph
