// eval_qd.hip -- quad-double values and Jacobian of gamma (1-t) g + t f
// (Eq. (1)) with the Jacobian row of the equation in flight held on chip, for
// the systems of the fast-path records (n <= 32, terms of at most 8 factors,
// exponents whose powers fit the LDS power table).
//
// A quad-double Jacobian row is 32 columns x 8 doubles per point, twice what
// the 256 accumulation registers of a lane hold.  So a point takes two
// adjacent lanes: lane 2p holds the real parts and lane 2p+1 the imaginary
// parts of point p, and each lane keeps its component of the row (32 columns
// x 4 limbs = 256 dwords) in the accumulation registers, column j in
// a[8j .. 8j+7], at one wave per SIMD as in the double-double kernel.  A wave
// covers 32 points.
//
// Every complex product is computed by both lanes of a point, each forming
// only its own component with one fused dot product (qd_dot2): with A held
// as "own" component in each lane, and B in natural form (re, im),
//     (A B)_own = A_own B_re + s A_other B_im,   s = -1 (real lane), +1 (imaginary lane),
// where A_other is the partner lane's own component (a DPP swap of adjacent
// lanes) and s is applied by flipping sign bits.  Coordinates and powers
// come from LDS in natural form (both lanes of a point read the same
// addresses); the suffix products, the only computed values used as B, are
// turned into natural form by a per-lane select of own and other.
//
// Per term the products are those of the other fast paths (Section 1
// decomposition, Table 6): c(t), times x^(a-1) for the factors with a >= 2
// (from the power table), the suffix products, and one forward pass issuing
// each partial beside the next prefix product.  A partial is added into the
// lane's row component with one fused update (qd_axpy).  H and J leave the
// kernel once per equation.
#include <hip/hip_runtime.h>

#include "ph_arith.hpp"
#include "ph_arow.hpp"
#include "ph_internal.hpp"

namespace ph {

struct QDArgs {
    const double *t;
    const double *x;
    double *val;
    double *jac;
    int64_t npts, ld;
    double gre, gim;
    int n_eq, n_var, eq_stride, planes;
};

// r + e * p in quad double with one renormalisation: TwoProd of e with the
// three leading limbs of p, the limbs and product errors summed level by
// level (TwoSum chains at levels 0..2, errors one level down, level 3 in
// plain FP64), as in qd_dot2.  e is a small integer exponent.
__device__ __forceinline__ R<4> qd_axpy(const R<4> &r, double e, const R<4> &p)
{
    double P0, E0, P1, E1, P2, E2;
    two_prod(e, p.v[0], P0, E0);
    two_prod(e, p.v[1], P1, E1);
    two_prod(e, p.v[2], P2, E2);
    double s0, t0;
    two_sum(r.v[0], P0, s0, t0);
    double s1, u1, u2, u3;
    two_sum(r.v[1], P1, s1, u1);
    two_sum(s1, E0, s1, u2);
    two_sum(s1, t0, s1, u3);
    double s2, w1, w2, w3, w4, w5;
    two_sum(r.v[2], P2, s2, w1);
    two_sum(s2, E1, s2, w2);
    two_sum(s2, u1, s2, w3);
    two_sum(s2, u2, s2, w4);
    two_sum(s2, u3, s2, w5);
    double s3 = __builtin_fma(e, p.v[3], r.v[3]);
    s3 += E2 + ((w1 + w2) + (w3 + w4)) + w5;
    return qd_renorm_safe(s0, s1, s2, s3, 0.0);
}

// the partner lane's value (the other component of the same point).  Every
// lane has a source lane in this permutation, so the move carries no "old"
// operand (which would cost a register set to zero per move)
__device__ __forceinline__ double pair_swap(double v)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, 0xB1, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), 0xB1, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// s * (partner's own component): the sign bit flipped in the real lane
// (sg = 0x80000000 there, 0 in the imaginary lane)
__device__ __forceinline__ R<4> other_signed(const R<4> &own, unsigned sg)
{
    R<4> r;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        const unsigned long long b = __builtin_bit_cast(unsigned long long, pair_swap(own.v[l]));
        r.v[l] = __builtin_bit_cast(double, b ^ ((unsigned long long)sg << 32));
    }
    return r;
}

// own component of A * B, A as (own, signed other), B natural
__device__ __forceinline__ R<4> pmul(const R<4> &aown, const R<4> &aoth_s, const C<4> &b)
{
    return qd_dot2(aown, b.re, aoth_s, b.im);
}

// LDS staging rows: ((plane * n + v) * 8 + 4 * comp + limb) * 32 + point;
// off = byte offset of the (plane, v) block (2048 bytes each)
__device__ __forceinline__ C<4> lds_nat(const char *__restrict__ xb, uint32_t off, int p)
{
    const double *q = reinterpret_cast<const double *>(xb + off) + p;
    C<4> z;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        z.re.v[l] = q[l * 32];
        z.im.v[l] = q[(4 + l) * 32];
    }
    return z;
}

// natural form of a computed value from its own and (unsigned) other component
__device__ __forceinline__ C<4> natural(const R<4> &own, const R<4> &oth, int c)
{
    C<4> z;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        z.re.v[l] = c ? oth.v[l] : own.v[l];
        z.im.v[l] = c ? own.v[l] : oth.v[l];
    }
    return z;
}

__device__ __forceinline__ void qrow_axpy(ARow &row, uint32_t jo, double e, const R<4> &part)
{
    R<4> r;
    row.read(jo, r.v[0], r.v[1], r.v[2], r.v[3]);
    r = qd_axpy(r, e, part);
    row.write(jo, r.v[0], r.v[1], r.v[2], r.v[3]);
}

// Per-point context of a lane.
struct QLane {
    int p, c;        // point within the tile, component (0 real, 1 imaginary)
    unsigned sg;     // sign mask of the product rule
    double tv;       // t
    R<4> gs_own, gs_oth_s;  // gamma (1 - t), own and signed other component
};

__device__ __forceinline__ R<4> qcoef(const MHead<4> &h, const QLane &ql)
{
    R<4> cre, cim;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        cre.v[l] = h.c[l];
        cim.v[l] = h.c[4 + l];
    }
    if (h.sel & 1) return qd_dot2(ql.gs_own, cre, ql.gs_oth_s, cim);  // gamma (1-t) c
    R<4> own;
#pragma unroll
    for (int l = 0; l < 4; ++l) own.v[l] = ql.c ? cim.v[l] : cre.v[l];
    return r_mul_d<4>(own, ql.tv);  // t c
}

// One term with K factors, the first M of them with a >= 2.
// (A quad-double term takes thousands of instructions, so its record is
// simply read at its start: the scalar loads are not on the critical path.)
template <int K, int M>
__device__ __forceinline__ void qfast_sweep(const MHead<4> &h, const char *__restrict__ xb, const QLane &ql,
                                            R<4> cf, ARow &row, R<4> &v)
{
    // common factor: c(t) times the powers x^(a-1), one product each
#pragma unroll
    for (int l = 0; l < M; ++l) {
        const C<4> pw = lds_nat(xb, h.po[l], ql.p);
        cf = pmul(cf, other_signed(cf, ql.sg), pw);
    }
    // suffix products sf[l] = x_l ... x_{K-1}, kept in natural form
    C<4> sfn[K > 1 ? K : 1];
    if constexpr (K > 1) {
        sfn[K - 1] = lds_nat(xb, h.xo[K - 1], ql.p);
        R<4> own = ql.c ? sfn[K - 1].im : sfn[K - 1].re;
        R<4> oth = ql.c ? sfn[K - 1].re : sfn[K - 1].im;
#pragma unroll
        for (int l = K - 2; l >= 1; --l) {
            const C<4> xl = lds_nat(xb, h.xo[l], ql.p);
            R<4> oth_s;
#pragma unroll
            for (int z = 0; z < 4; ++z)
                oth_s.v[z] = __builtin_bit_cast(double, __builtin_bit_cast(unsigned long long, oth.v[z]) ^
                                                           ((unsigned long long)ql.sg << 32));
            own = pmul(own, oth_s, xl);
#pragma unroll
            for (int z = 0; z < 4; ++z) oth.v[z] = pair_swap(own.v[z]);
            sfn[l] = natural(own, oth, ql.c);
        }
    }
    // forward pass: q = cf x_0 ... x_{l-1}; partial l = q sf[l+1]
    R<4> q = cf;
#pragma unroll
    for (int l = 0; l < K - 1; ++l) {
        const R<4> qo = other_signed(q, ql.sg);
        const R<4> part = pmul(q, qo, sfn[l + 1]);
        q = pmul(q, qo, lds_nat(xb, h.xo[l], ql.p));
        qrow_axpy(row, h.jo[l], h.a[l], part);
    }
    v = r_add<4>(v, pmul(q, other_signed(q, ql.sg), lds_nat(xb, h.xo[K - 1], ql.p)));
    qrow_axpy(row, h.jo[K - 1], h.a[K - 1], q);
}

template <int K, int M, int KF>
__device__ __forceinline__ void qfast_groups(const int32_t *__restrict__ run, const MTerm *__restrict__ mt,
                                             const char *__restrict__ xb, const QLane &ql, ARow &row, R<4> &v)
{
    constexpr int g = drun_group(K, M);
    const int s0 = run[g], s1 = run[g + 1];
    for (int s = s0; s < s1; ++s) {
        const MHead<4> h = mfast_head<K, M, 4>(mt + s);
        qfast_sweep<K, M>(h, xb, ql, qcoef(h, ql), row, v);
    }
    if constexpr (M < K)
        qfast_groups<K, M + 1, KF>(run, mt, xb, ql, row, v);
    else if constexpr (K < KF)
        qfast_groups<K + 1, 0, KF>(run, mt, xb, ql, row, v);
}

__device__ __forceinline__ void st_nt4(double *p, double v) { __builtin_nontemporal_store(v, p); }

// One wave per SIMD (256 architectural registers for the sweep, 256 AGPRs
// for the row component); at most four waves per workgroup.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
eval_qd_arow_kernel(QDArgs a, const int32_t *__restrict__ d_run, const MTerm *__restrict__ mterm,
                    const int32_t *__restrict__ d_deg)
{
    extern __shared__ double xl[];
    const char *xb = reinterpret_cast<const char *>(xl);
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int W = blockDim.x >> 6;
    QLane ql;
    ql.p = lane >> 1;
    ql.c = lane & 1;
    ql.sg = ql.c ? 0u : 0x80000000u;
    const int64_t P = (int64_t)blockIdx.x * 32 + ql.p;
    const bool act = P < a.npts;
    const int nv = a.n_var;
    // stage x and its powers (each lane writes its component's four rows)
    for (int var = w; var < nv; var += W) {
        C<4> x1 = c_zero<4>();
        if (act) {
#pragma unroll
            for (int l = 0; l < 4; ++l) {
                x1.re.v[l] = a.x[(int64_t)(var * 8 + l) * a.ld + P];
                x1.im.v[l] = a.x[(int64_t)(var * 8 + 4 + l) * a.ld + P];
            }
        }
        C<4> z = x1;
        for (int q = 0; q < a.planes; ++q) {
            double *row = xl + (size_t)((q * nv + var) * 8 + 4 * ql.c) * 32 + ql.p;
            const R<4> own = ql.c ? z.im : z.re;
#pragma unroll
            for (int l = 0; l < 4; ++l) row[l * 32] = own.v[l];
            if (q + 1 < a.planes) z = c_mul<4>(z, x1);
        }
    }
    if (w == 0) {
        double *row = xl + (size_t)(a.planes * nv * 8 + 4 * ql.c) * 32 + ql.p;
#pragma unroll
        for (int l = 0; l < 4; ++l) row[l * 32] = (ql.c == 0 && l == 0) ? 1.0 : 0.0;
    }
    __syncthreads();

    // c(t): t for target terms, gamma (1 - t) for start terms, (1 - t) exact
    ql.tv = 1.0;
    if (a.t) ql.tv = act ? a.t[P] : 0.0;
    C<4> gs = c_zero<4>();
    if (a.t) {
        double o, oe;
        two_sum(1.0, -ql.tv, o, oe);
        R<4> omt = r_zero<4>();
        omt.v[0] = o;
        omt.v[1] = oe;
        gs = c_mul_r<4>(c_from<4>(a.gre, a.gim), omt);
    }
    ql.gs_own = ql.c ? gs.im : gs.re;
    {
        const R<4> oth = ql.c ? gs.re : gs.im;
#pragma unroll
        for (int l = 0; l < 4; ++l)
            ql.gs_oth_s.v[l] = __builtin_bit_cast(double, __builtin_bit_cast(unsigned long long, oth.v[l]) ^
                                                              ((unsigned long long)ql.sg << 32));
    }

    for (int i = blockIdx.y * W + w; i < a.n_eq; i += a.eq_stride) {
        ARow row;
        row.zero();
        R<4> v = r_zero<4>();
        const int32_t *run = d_run + i * DRUN;
        for (int s = run[0]; s < run[1]; ++s) v = r_add<4>(v, qcoef(mfast_head<0, 0, 4>(mterm + s), ql));
        qfast_groups<1, 0, 8>(run, mterm, xb, ql, row, v);
        // total-degree start part: gamma (1-t) (x_i^d - 1), derivative d x_i^(d-1)
        // (whole complex values in both lanes, then the own component)
        const int d = d_deg[i];
        if (d > 0 && a.t) {
            const C<4> xi = lds_nat(xb, (uint32_t)(i * 2048), ql.p);
            C<4> pw = c_from<4>(1.0, 0.0), base = xi;  // pw = x_i^(d-1)
            for (int e = d - 1; e > 0; e >>= 1) {
                if (e & 1) pw = c_mul<4>(pw, base);
                if (e > 1) base = c_mul<4>(base, base);
            }
            const C<4> gp = c_mul<4>(gs, pw);
            const C<4> hv = c_sub<4>(c_mul<4>(gp, xi), gs);
            v = r_add<4>(v, ql.c ? hv.im : hv.re);
            qrow_axpy(row, (uint32_t)(8 * i), (double)d, ql.c ? gp.im : gp.re);
        }
        if (act) {
            double *hp = a.val + (int64_t)((i * 2 + ql.c) * 4) * a.ld + P;
#pragma unroll
            for (int l = 0; l < 4; ++l) st_nt4(hp + l * a.ld, v.v[l]);
            double *jr = a.jac + (int64_t)((i * nv * 2 + ql.c) * 4) * a.ld + P;
            for (int j = 0; j < nv; ++j) {
                R<4> r;
                row.read((uint32_t)(8 * j), r.v[0], r.v[1], r.v[2], r.v[3]);
                double *q = jr + (int64_t)(j * 8) * a.ld;
#pragma unroll
                for (int l = 0; l < 4; ++l) st_nt4(q + l * a.ld, r.v[l]);
            }
        }
    }
}

int qd_fast_launch(const DevTable &tab, const double gamma[2], int64_t npts, const double *t,
                   const double *x, int64_t ld, double *val, double *jac, int W, int G,
                   hipStream_t st)
{
    QDArgs a;
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
    const size_t lds = ((size_t)tab.dfast_planes * tab.n_var * 8 + 8) * 32 * sizeof(double);
    dim3 grid((unsigned)((npts + 31) / 32), (unsigned)G);
    hipLaunchKernelGGL(eval_qd_arow_kernel, grid, dim3(64 * W), lds, st, a, tab.d_run, tab.mterm, tab.d_deg);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "eval_qd_arow_kernel launch");
    return PH_OK;
}

}  // namespace ph
