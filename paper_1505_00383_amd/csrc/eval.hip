// eval.hip -- values and Jacobian of gamma (1-t) g(x) + t f(x) at many points
// (Eq. (1) of the paper), the evaluation stage of Section 2 and the kernels of
// Section 3 (coefficients c(t), monomials by reverse mode, sums) fused into one.
//
// Mapping onto gfx950:
//   * one lane = one point; a wave runs the merged term stream of one
//     equation on 64 points at once, so every term index, exponent and
//     coefficient is wave-uniform and comes through scalar loads (Section 3:
//     all threads of a block evaluate the same monomial at different points);
//   * all waves of a workgroup work on the same 64 points, each on its own
//     equations, and share the coordinates staged once in LDS in the layout
//     [row][lane] (row = (var*2+c)*L + l), which is conflict-free for a wave;
//   * point data in HBM is structure-of-arrays with the point index fastest
//     (the transposed layout of Table 5), so every global access of a wave is
//     one contiguous 512-byte segment;
//   * the Jacobian row of the equation in flight is accumulated in place in
//     the output array (L2-resident during the equation); the first
//     contribution to a column is a store, columns no term touches get a zero.
//
// Per term c * prod_l x_{j_l}^{a_l} (Section 1 decomposition, Table 6):
//   cf   = c(t) * prod_l x_{j_l}^{a_l - 1}         common factor
//   q_l  = cf * x_{j_1} ... x_{j_{l-1}}           forward products
//   value = q_k * x_{j_k}
//   d/dx_{j_l} = a_l * q_l * (x_{j_{l+1}} ... x_{j_k})   backward products
// which is 3k - 3 products including the two that fold cf in (3k - 5 for the
// bare variable product, as counted in Table 6).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "ph_arith.hpp"
#include "ph_internal.hpp"
#include "ph_sweep.hpp"

namespace ph {

struct EvalArgs {
    const int32_t *eq_off;
    const int4 *tdesc;
    const uint32_t *fac;
    const double *coef;
    const int32_t *zc_off;
    const int32_t *zc;
    const double *t;
    const double *x;
    double *val;
    double *jac;
    int64_t npts, ld;
    double gre, gim;
    int n_eq, n_var, eq_stride;
};

template <int L>
__device__ __forceinline__ C<L> load_x(const double *__restrict__ xl, int var, int lane)
{
    C<L> z;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        z.re.v[l] = xl[((var * 2 + 0) * L + l) * 64 + lane];
        z.im.v[l] = xl[((var * 2 + 1) * L + l) * 64 + lane];
    }
    return z;
}

template <int L>
__device__ __forceinline__ C<L> load_x_global(const double *__restrict__ x, int var, int64_t ld,
                                              int64_t p)
{
    C<L> z;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        z.re.v[l] = x[((int64_t)(var * 2 + 0) * L + l) * ld + p];
        z.im.v[l] = x[((int64_t)(var * 2 + 1) * L + l) * ld + p];
    }
    return z;
}

// Add (or store, on the first touch) one partial derivative into the output.
template <int L>
__device__ __forceinline__ void jac_acc(double *__restrict__ jrow, int64_t ld, bool first, C<L> d,
                                        bool act)
{
    if (!act) return;
    if (first) {
#pragma unroll
        for (int l = 0; l < L; ++l) {
            jrow[(int64_t)l * ld] = d.re.v[l];
            jrow[(int64_t)(L + l) * ld] = d.im.v[l];
        }
    } else {
        C<L> o;
#pragma unroll
        for (int l = 0; l < L; ++l) {
            o.re.v[l] = jrow[(int64_t)l * ld];
            o.im.v[l] = jrow[(int64_t)(L + l) * ld];
        }
        o = c_add<L>(o, d);
#pragma unroll
        for (int l = 0; l < L; ++l) {
            jrow[(int64_t)l * ld] = o.re.v[l];
            jrow[(int64_t)(L + l) * ld] = o.im.v[l];
        }
    }
}

template <int L, int KMAX, bool XLDS, bool JAC>
__device__ __forceinline__ void eval_body(const EvalArgs &a)
{
    extern __shared__ double xl[];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int W = blockDim.x >> 6;
    const int64_t p = (int64_t)blockIdx.x * 64 + lane;
    const bool act = p < a.npts;
    const int nv = a.n_var;

    if constexpr (XLDS) {
        const int rows = nv * 2 * L;
        for (int r = w; r < rows; r += W) xl[r * 64 + lane] = act ? a.x[(int64_t)r * a.ld + p] : 0.0;
        __syncthreads();
    }
    auto X = [&](int var) -> C<L> {
        if constexpr (XLDS)
            return load_x<L>(xl, var, lane);
        else
            return act ? load_x_global<L>(a.x, var, a.ld, p) : c_zero<L>();
    };

    // c(t) per point: t for target terms, gamma (1 - t) for start terms;
    // (1 - t) is exact in two limbs.
    double tv = 1.0;
    if (a.t) tv = act ? a.t[p] : 0.0;
    C<L> gs = c_zero<L>();
    if (a.t) {
        double o, oe;
        two_sum(1.0, -tv, o, oe);
        R<L> omt = r_zero<L>();
        omt.v[0] = o;
        if constexpr (L > 1) omt.v[1] = oe;
        gs = c_mul_r<L>(c_from<L>(a.gre, a.gim), omt);
    }

    for (int i = blockIdx.y * W + w; i < a.n_eq; i += a.eq_stride) {
        C<L> v = c_zero<L>();
        double *jrow0 = JAC ? a.jac + (int64_t)i * nv * 2 * L * a.ld + p : nullptr;
        const int s0 = a.eq_off[i], s1 = a.eq_off[i + 1];
        for (int s = s0; s < s1; ++s) {
            const int4 d = a.tdesc[s];
            const int k = d.x;
            C<L> c;
#pragma unroll
            for (int l = 0; l < L; ++l) {
                c.re.v[l] = a.coef[(int64_t)s * 8 + l];
                c.im.v[l] = a.coef[(int64_t)s * 8 + 4 + l];
            }
            c = d.z ? c_mul<L>(c, gs) : c_mul_d<L>(c, tv);
            if (k == 0) {
                v = c_add<L>(v, c);
                continue;
            }
            uint32_t fw[KMAX];
#pragma unroll
            for (int l = 0; l < KMAX; ++l)
                if (l < k) fw[l] = a.fac[d.y + l];
            const C<L> tv_term = term_sweep<KMAX, JAC, (L == 1)>(
                k, fw, c, X, [&](int, uint32_t w, const C<L> &part) {
                    if constexpr (JAC)
                        jac_acc<L>(jrow0 + (int64_t)fac_var(w) * 2 * L * a.ld, a.ld,
                                   (w & FAC_FIRST) != 0, part, act);
                });
            v = c_add<L>(v, tv_term);
        }
        if (act) {
#pragma unroll
            for (int l = 0; l < L; ++l) {
                a.val[((int64_t)(i * 2 + 0) * L + l) * a.ld + p] = v.re.v[l];
                a.val[((int64_t)(i * 2 + 1) * L + l) * a.ld + p] = v.im.v[l];
            }
            if constexpr (JAC) {
                for (int z = a.zc_off[i]; z < a.zc_off[i + 1]; ++z) {
                    double *jr = jrow0 + (int64_t)a.zc[z] * 2 * L * a.ld;
#pragma unroll
                    for (int l = 0; l < 2 * L; ++l) jr[(int64_t)l * a.ld] = 0.0;
                }
            }
        }
    }
}

template <int L, int KMAX, bool XLDS, bool JAC>
__global__ void __launch_bounds__(512) eval_kernel(EvalArgs a)
{
    eval_body<L, KMAX, XLDS, JAC>(a);
}

// The same at one wave per SIMD (at most four waves per workgroup): the
// quad-double sweep then has 512 registers and spills nothing to scratch.
template <int L, int KMAX, bool XLDS, bool JAC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) eval_kernel_w1(EvalArgs a)
{
    eval_body<L, KMAX, XLDS, JAC>(a);
}

// H and J leave a register-row kernel exactly once and are not read again by
// it: non-temporal stores stream them to HBM instead of keeping them in the
// caches (about 11 % more write bandwidth on the write-bound workloads).
__device__ __forceinline__ void st_out(double *p, double v) { __builtin_nontemporal_store(v, p); }

// ---------------------------------------------------------------------------
// Complex double with n_var <= 32: the Jacobian row of the equation in flight
// stays in registers.  The row is four 32-entry planes (low/high 32 bits of
// the real and imaginary parts) so that a wave-uniform column index addresses
// it through the GPR indexing mode (s_set_gpr_idx_on) without any branch:
// four indexed moves in, two adds, four indexed moves out per partial.
// ---------------------------------------------------------------------------
typedef unsigned int v32u __attribute__((ext_vector_type(32)));

struct RegRow {
    v32u rl, rh, il, ih;
};

__device__ __forceinline__ void regrow_add(RegRow &r, int j, const C<1> &d)
{
    const unsigned long long a = ((unsigned long long)r.rh[j] << 32) | r.rl[j];
    const unsigned long long b = ((unsigned long long)r.ih[j] << 32) | r.il[j];
    const double x = __builtin_bit_cast(double, a) + d.re.v[0];
    const double y = __builtin_bit_cast(double, b) + d.im.v[0];
    const unsigned long long xa = __builtin_bit_cast(unsigned long long, x);
    const unsigned long long yb = __builtin_bit_cast(unsigned long long, y);
    r.rl[j] = (unsigned)xa;
    r.rh[j] = (unsigned)(xa >> 32);
    r.il[j] = (unsigned)yb;
    r.ih[j] = (unsigned)(yb >> 32);
}

template <int KMAX>
__global__ void __launch_bounds__(512) eval_d_regrow_kernel(EvalArgs a)
{
    extern __shared__ double xl[];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int W = blockDim.x >> 6;
    const int64_t p = (int64_t)blockIdx.x * 64 + lane;
    const bool act = p < a.npts;
    const int nv = a.n_var;
    const int rows = nv * 2;
    for (int r = w; r < rows; r += W) xl[r * 64 + lane] = act ? a.x[(int64_t)r * a.ld + p] : 0.0;
    __syncthreads();
    auto X = [&](int var) -> C<1> { return load_x<1>(xl, var, lane); };

    double tv = 1.0;
    if (a.t) tv = act ? a.t[p] : 0.0;
    C<1> gs = c_zero<1>();
    if (a.t) gs = c_mul_d<1>(c_from<1>(a.gre, a.gim), 1.0 - tv);

    for (int i = blockIdx.y * W + w; i < a.n_eq; i += a.eq_stride) {
        RegRow row;
        row.rl = 0;
        row.rh = 0;
        row.il = 0;
        row.ih = 0;
        C<1> v = c_zero<1>();
        const int s0 = a.eq_off[i], s1 = a.eq_off[i + 1];
        for (int s = s0; s < s1; ++s) {
            const int4 d = a.tdesc[s];
            const int k = d.x;
            C<1> c = c_from<1>(a.coef[(int64_t)s * 8], a.coef[(int64_t)s * 8 + 4]);
            c = d.z ? c_mul<1>(c, gs) : c_mul_d<1>(c, tv);
            if (k == 0) {
                v = c_add<1>(v, c);
                continue;
            }
            uint32_t fw[KMAX];
#pragma unroll
            for (int l = 0; l < KMAX; ++l)
                if (l < k) fw[l] = __builtin_amdgcn_readfirstlane(a.fac[d.y + l]);
            v = c_add<1>(v, term_sweep<KMAX, true, false>(k, fw, c, X,
                                                   [&](int, uint32_t wd, const C<1> &part) {
                                                       regrow_add(row, fac_var(wd), part);
                                                   }));
        }
        if (act) {
            st_out(&a.val[((int64_t)(i * 2 + 0)) * a.ld + p], v.re.v[0]);
            st_out(&a.val[((int64_t)(i * 2 + 1)) * a.ld + p], v.im.v[0]);
            double *jr = a.jac + (int64_t)i * nv * 2 * a.ld + p;
#pragma unroll
            for (int j = 0; j < 32; ++j) {
                if (j < nv) {
                    st_out(&jr[(int64_t)(j * 2 + 0) * a.ld],
                           __builtin_bit_cast(double, ((unsigned long long)row.rh[j] << 32) | row.rl[j]));
                    st_out(&jr[(int64_t)(j * 2 + 1) * a.ld],
                           __builtin_bit_cast(double, ((unsigned long long)row.ih[j] << 32) | row.il[j]));
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Complex-double fast path (terms with k <= 8 factors and exponents <= 4):
// per-point powers x, x^2, x^3 and a row of ones are staged in LDS, so the
// common factor is k branch-free products by x^(a_l - 1); each k has its own
// fully unrolled sweep; the exponent a_l rides in the FMA that adds the
// partial into the register-resident Jacobian row; the total-degree start
// part gamma (1-t) (x_i^d - 1) is evaluated once per equation by binary
// powering.
// ---------------------------------------------------------------------------
__device__ __forceinline__ C<1> ldsc(const char *__restrict__ xb, uint32_t off, int lane)
{
    const double *p = reinterpret_cast<const double *>(xb + off);
    return c_from<1>(p[lane], p[64 + lane]);
}

// row[j] += q * d (complex) as four FMAs into the row entry
__device__ __forceinline__ void regrow_cfma(RegRow &r, int j, const C<1> &q, const C<1> &d)
{
    const unsigned long long a = ((unsigned long long)r.rh[j] << 32) | r.rl[j];
    const unsigned long long b = ((unsigned long long)r.ih[j] << 32) | r.il[j];
    double x = __builtin_fma(q.re.v[0], d.re.v[0], __builtin_bit_cast(double, a));
    double y = __builtin_fma(q.re.v[0], d.im.v[0], __builtin_bit_cast(double, b));
    x = __builtin_fma(-q.im.v[0], d.im.v[0], x);
    y = __builtin_fma(q.im.v[0], d.re.v[0], y);
    const unsigned long long xa = __builtin_bit_cast(unsigned long long, x);
    const unsigned long long yb = __builtin_bit_cast(unsigned long long, y);
    r.rl[j] = (unsigned)xa;
    r.rh[j] = (unsigned)(xa >> 32);
    r.il[j] = (unsigned)yb;
    r.ih[j] = (unsigned)(yb >> 32);
}

__device__ __forceinline__ void regrow_fma(RegRow &r, int j, double e, const C<1> &d)
{
    const unsigned long long a = ((unsigned long long)r.rh[j] << 32) | r.rl[j];
    const unsigned long long b = ((unsigned long long)r.ih[j] << 32) | r.il[j];
    const double x = __builtin_fma(e, d.re.v[0], __builtin_bit_cast(double, a));
    const double y = __builtin_fma(e, d.im.v[0], __builtin_bit_cast(double, b));
    const unsigned long long xa = __builtin_bit_cast(unsigned long long, x);
    const unsigned long long yb = __builtin_bit_cast(unsigned long long, y);
    r.rl[j] = (unsigned)xa;
    r.rh[j] = (unsigned)(xa >> 32);
    r.il[j] = (unsigned)yb;
    r.ih[j] = (unsigned)(yb >> 32);
}

// The same row held by the compiler (four indexed planes, see RegRow).
struct VecRow {
    static constexpr bool kIndexed = false;  // columns addressed by compile-time index
    RegRow r;
    __device__ __forceinline__ void zero()
    {
        r.rl = 0;
        r.rh = 0;
        r.il = 0;
        r.ih = 0;
    }
    __device__ __forceinline__ void fma(int j2, double e, const C<1> &d) { regrow_fma(r, j2 >> 1, e, d); }
    __device__ __forceinline__ void cfma(int j2, const C<1> &q, const C<1> &d) { regrow_cfma(r, j2 >> 1, q, d); }
    __device__ __forceinline__ void get(int j, double &re, double &im)
    {
        re = __builtin_bit_cast(double, ((unsigned long long)r.rh[j] << 32) | r.rl[j]);
        im = __builtin_bit_cast(double, ((unsigned long long)r.ih[j] << 32) | r.il[j]);
    }
};

// The row pinned in the upper half of the register file: real parts of
// columns 0..31 in v[128:191], imaginary parts in v[192:255].  The kernel is
// compiled with a 128-register budget, so the compiler never allocates these
// registers; every statement that touches them lists all of them as
// clobbered (which also makes the kernel descriptor reserve 256 registers).
// A partial is added with the column index applied by the GPR indexing mode
// to the destination and addend of two FP64 FMAs: no register moves at all.
// s_set_gpr_idx_on writes the index into M0.  The compiler reserves M0 and
// does not honour it in a clobber list, so instead the compiled pinned
// kernels are checked to contain no compiler-generated instruction that uses
// M0 at all (no value of the compiler's can live in M0 across these blocks).
// fma takes twice the column index; callers guarantee 0 <= j < 32 (the fast
// path requires n_var <= 32).
#define PH_PIN_CLOBBERS "v128","v129","v130","v131","v132","v133","v134","v135","v136","v137","v138","v139","v140","v141","v142","v143","v144","v145","v146","v147","v148","v149","v150","v151","v152","v153","v154","v155","v156","v157","v158","v159","v160","v161","v162","v163","v164","v165","v166","v167","v168","v169","v170","v171","v172","v173","v174","v175","v176","v177","v178","v179","v180","v181","v182","v183","v184","v185","v186","v187","v188","v189","v190","v191","v192","v193","v194","v195","v196","v197","v198","v199","v200","v201","v202","v203","v204","v205","v206","v207","v208","v209","v210","v211","v212","v213","v214","v215","v216","v217","v218","v219","v220","v221","v222","v223","v224","v225","v226","v227","v228","v229","v230","v231","v232","v233","v234","v235","v236","v237","v238","v239","v240","v241","v242","v243","v244","v245","v246","v247","v248","v249","v250","v251","v252","v253","v254","v255"
struct PinRow {
    static constexpr bool kIndexed = true;  // any column by the GPR index mode
    __device__ __forceinline__ void zero()
    {
        asm volatile("v_mov_b64 v[128:129], 0\n\tv_mov_b64 v[130:131], 0\n\tv_mov_b64 v[132:133], 0\n\tv_mov_b64 v[134:135], 0\n\tv_mov_b64 v[136:137], 0\n\tv_mov_b64 v[138:139], 0\n\tv_mov_b64 v[140:141], 0\n\tv_mov_b64 v[142:143], 0\n\tv_mov_b64 v[144:145], 0\n\tv_mov_b64 v[146:147], 0\n\tv_mov_b64 v[148:149], 0\n\tv_mov_b64 v[150:151], 0\n\tv_mov_b64 v[152:153], 0\n\tv_mov_b64 v[154:155], 0\n\tv_mov_b64 v[156:157], 0\n\tv_mov_b64 v[158:159], 0\n\tv_mov_b64 v[160:161], 0\n\tv_mov_b64 v[162:163], 0\n\tv_mov_b64 v[164:165], 0\n\tv_mov_b64 v[166:167], 0\n\tv_mov_b64 v[168:169], 0\n\tv_mov_b64 v[170:171], 0\n\tv_mov_b64 v[172:173], 0\n\tv_mov_b64 v[174:175], 0\n\tv_mov_b64 v[176:177], 0\n\tv_mov_b64 v[178:179], 0\n\tv_mov_b64 v[180:181], 0\n\tv_mov_b64 v[182:183], 0\n\tv_mov_b64 v[184:185], 0\n\tv_mov_b64 v[186:187], 0\n\tv_mov_b64 v[188:189], 0\n\tv_mov_b64 v[190:191], 0\n\tv_mov_b64 v[192:193], 0\n\tv_mov_b64 v[194:195], 0\n\tv_mov_b64 v[196:197], 0\n\tv_mov_b64 v[198:199], 0\n\tv_mov_b64 v[200:201], 0\n\tv_mov_b64 v[202:203], 0\n\tv_mov_b64 v[204:205], 0\n\tv_mov_b64 v[206:207], 0\n\tv_mov_b64 v[208:209], 0\n\tv_mov_b64 v[210:211], 0\n\tv_mov_b64 v[212:213], 0\n\tv_mov_b64 v[214:215], 0\n\tv_mov_b64 v[216:217], 0\n\tv_mov_b64 v[218:219], 0\n\tv_mov_b64 v[220:221], 0\n\tv_mov_b64 v[222:223], 0\n\tv_mov_b64 v[224:225], 0\n\tv_mov_b64 v[226:227], 0\n\tv_mov_b64 v[228:229], 0\n\tv_mov_b64 v[230:231], 0\n\tv_mov_b64 v[232:233], 0\n\tv_mov_b64 v[234:235], 0\n\tv_mov_b64 v[236:237], 0\n\tv_mov_b64 v[238:239], 0\n\tv_mov_b64 v[240:241], 0\n\tv_mov_b64 v[242:243], 0\n\tv_mov_b64 v[244:245], 0\n\tv_mov_b64 v[246:247], 0\n\tv_mov_b64 v[248:249], 0\n\tv_mov_b64 v[250:251], 0\n\tv_mov_b64 v[252:253], 0\n\tv_mov_b64 v[254:255], 0" ::: PH_PIN_CLOBBERS);
    }
    __device__ __forceinline__ void fma(int j2, double e, const C<1> &d)
    {
        asm volatile("s_set_gpr_idx_on %0, gpr_idx(SRC2,DST)\n\t"
                     "v_fma_f64 v[128:129], %1, %2, v[128:129]\n\t"
                     "v_fma_f64 v[192:193], %1, %3, v[192:193]\n\t"
                     "s_set_gpr_idx_off"
                     :
                     : "s"(j2), "s"(e), "v"(d.re.v[0]), "v"(d.im.v[0])
                     : PH_PIN_CLOBBERS);
    }
    // row[j] += q * d (complex): four FMAs into the row, the product never
    // rounded on its own (a factor with exponent 1 needs no scaling)
    __device__ __forceinline__ void cfma(int j2, const C<1> &q, const C<1> &d)
    {
        asm volatile("s_set_gpr_idx_on %0, gpr_idx(SRC2,DST)\n\t"
                     "v_fma_f64 v[128:129], %1, %3, v[128:129]\n\t"
                     "v_fma_f64 v[192:193], %1, %4, v[192:193]\n\t"
                     "v_fma_f64 v[128:129], -%2, %4, v[128:129]\n\t"
                     "v_fma_f64 v[192:193], %2, %3, v[192:193]\n\t"
                     "s_set_gpr_idx_off"
                     :
                     : "s"(j2), "v"(q.re.v[0]), "v"(q.im.v[0]), "v"(d.re.v[0]), "v"(d.im.v[0])
                     : PH_PIN_CLOBBERS);
    }
    __device__ __forceinline__ void get(int j, double &re, double &im)
    {
        unsigned rl, rh, il, ih;
        asm volatile("s_set_gpr_idx_on %4, gpr_idx(SRC0)\n\t"
                     "v_mov_b32 %0, v128\n\t"
                     "v_mov_b32 %1, v129\n\t"
                     "v_mov_b32 %2, v192\n\t"
                     "v_mov_b32 %3, v193\n\t"
                     "s_set_gpr_idx_off"
                     : "=v"(rl), "=v"(rh), "=v"(il), "=v"(ih)
                     : "s"(2 * j)
                     : PH_PIN_CLOBBERS);
        re = __builtin_bit_cast(double, ((unsigned long long)rh << 32) | rl);
        im = __builtin_bit_cast(double, ((unsigned long long)ih << 32) | il);
    }
};

// The row of a system with at most 16 unknowns, pinned in v[64:127] (real
// parts of columns 0..15 in v[64:95], imaginary parts in v[96:127]) for a
// kernel compiled with a 64-register budget: 128 registers in all, so four
// waves fit each SIMD instead of two.  Same rules as PinRow.
#define PH_PIN16_CLOBBERS "v64","v65","v66","v67","v68","v69","v70","v71","v72","v73","v74","v75","v76","v77","v78","v79","v80","v81","v82","v83","v84","v85","v86","v87","v88","v89","v90","v91","v92","v93","v94","v95","v96","v97","v98","v99","v100","v101","v102","v103","v104","v105","v106","v107","v108","v109","v110","v111","v112","v113","v114","v115","v116","v117","v118","v119","v120","v121","v122","v123","v124","v125","v126","v127"
struct PinRow16 {
    static constexpr bool kIndexed = true;
    __device__ __forceinline__ void zero()
    {
        asm volatile("v_mov_b64 v[64:65], 0\n\tv_mov_b64 v[66:67], 0\n\tv_mov_b64 v[68:69], 0\n\tv_mov_b64 v[70:71], 0\n\tv_mov_b64 v[72:73], 0\n\tv_mov_b64 v[74:75], 0\n\tv_mov_b64 v[76:77], 0\n\tv_mov_b64 v[78:79], 0\n\tv_mov_b64 v[80:81], 0\n\tv_mov_b64 v[82:83], 0\n\tv_mov_b64 v[84:85], 0\n\tv_mov_b64 v[86:87], 0\n\tv_mov_b64 v[88:89], 0\n\tv_mov_b64 v[90:91], 0\n\tv_mov_b64 v[92:93], 0\n\tv_mov_b64 v[94:95], 0\n\tv_mov_b64 v[96:97], 0\n\tv_mov_b64 v[98:99], 0\n\tv_mov_b64 v[100:101], 0\n\tv_mov_b64 v[102:103], 0\n\tv_mov_b64 v[104:105], 0\n\tv_mov_b64 v[106:107], 0\n\tv_mov_b64 v[108:109], 0\n\tv_mov_b64 v[110:111], 0\n\tv_mov_b64 v[112:113], 0\n\tv_mov_b64 v[114:115], 0\n\tv_mov_b64 v[116:117], 0\n\tv_mov_b64 v[118:119], 0\n\tv_mov_b64 v[120:121], 0\n\tv_mov_b64 v[122:123], 0\n\tv_mov_b64 v[124:125], 0\n\tv_mov_b64 v[126:127], 0" ::: PH_PIN16_CLOBBERS);
    }
    __device__ __forceinline__ void fma(int j2, double e, const C<1> &d)
    {
        asm volatile("s_set_gpr_idx_on %0, gpr_idx(SRC2,DST)\n\t"
                     "v_fma_f64 v[64:65], %1, %2, v[64:65]\n\t"
                     "v_fma_f64 v[96:97], %1, %3, v[96:97]\n\t"
                     "s_set_gpr_idx_off"
                     :
                     : "s"(j2), "s"(e), "v"(d.re.v[0]), "v"(d.im.v[0])
                     : PH_PIN16_CLOBBERS);
    }
    __device__ __forceinline__ void cfma(int j2, const C<1> &q, const C<1> &d)
    {
        asm volatile("s_set_gpr_idx_on %0, gpr_idx(SRC2,DST)\n\t"
                     "v_fma_f64 v[64:65], %1, %3, v[64:65]\n\t"
                     "v_fma_f64 v[96:97], %1, %4, v[96:97]\n\t"
                     "v_fma_f64 v[64:65], -%2, %4, v[64:65]\n\t"
                     "v_fma_f64 v[96:97], %2, %3, v[96:97]\n\t"
                     "s_set_gpr_idx_off"
                     :
                     : "s"(j2), "v"(q.re.v[0]), "v"(q.im.v[0]), "v"(d.re.v[0]), "v"(d.im.v[0])
                     : PH_PIN16_CLOBBERS);
    }
    __device__ __forceinline__ void get(int j, double &re, double &im)
    {
        unsigned rl, rh, il, ih;
        asm volatile("s_set_gpr_idx_on %4, gpr_idx(SRC0)\n\t"
                     "v_mov_b32 %0, v64\n\t"
                     "v_mov_b32 %1, v65\n\t"
                     "v_mov_b32 %2, v96\n\t"
                     "v_mov_b32 %3, v97\n\t"
                     "s_set_gpr_idx_off"
                     : "=v"(rl), "=v"(rh), "=v"(il), "=v"(ih)
                     : "s"(2 * j)
                     : PH_PIN16_CLOBBERS);
        re = __builtin_bit_cast(double, ((unsigned long long)rh << 32) | rl);
        im = __builtin_bit_cast(double, ((unsigned long long)ih << 32) | il);
    }
};

// Scalar copy of a record: everything the sweep reads, fetched one term
// ahead so that no scalar load is waited for inside a term.
struct DHead {
    double cre, cim;
    int sel;
    uint32_t xo[8], po[8], j2[8];
    double a[8];
};

template <int K, int M>
__device__ __forceinline__ DHead dfast_head(const DTerm *__restrict__ r)
{
    DHead h;
    h.cre = r->cre;
    h.cim = r->cim;
    h.sel = r->sel;
#pragma unroll
    for (int l = 0; l < K; ++l) h.xo[l] = r->xo[l];
#pragma unroll
    for (int l = 0; l < M; ++l) h.po[l] = r->po[l];
#pragma unroll
    for (int l = 0; l < K; ++l) h.j2[l] = r->j2[l];
#pragma unroll
    for (int l = 0; l < K; ++l) h.a[l] = r->a[l];
    return h;
}

// One term with exactly K factors, the first M of them with exponent >= 2
// (the host sorts factors by exponent and groups records by (K, M)), with
// the products of Table 6 reordered for instruction-level parallelism: all
// coordinates and powers are read from LDS first, and the head of the NEXT
// record (same group) is fetched right after; the suffix products
// x_l ... x_{K-1} do not depend on the common factor and form a chain of
// their own; the M powers x^(a-1) are multiplied into the coefficient by a
// balanced tree; then one forward pass carries the running prefix product
// and issues, at each factor, the cross product with the suffix beside the
// next prefix product, so that only one prefix product is ever live.
// 3K - 3 + M complex products, the cost model's count (the cross products
// of the K - M factors with exponent 1 are fused into their row updates).
// A term's factors are distinct unknowns, so the order of its row updates
// does not change any result.
template <int K, int M, class Row>
__device__ __forceinline__ void dfast_sweep(const DHead &h, const DTerm *__restrict__ rnext, DHead &hnext,
                                            const char *__restrict__ xb, int lane, C<1> cf,
                                            Row &row, C<1> &v)
{
    C<1> xv[K], pw[M > 0 ? M : 1], sf[K];
#pragma unroll
    for (int l = 0; l < K; ++l) xv[l] = ldsc(xb, h.xo[l], lane);
    // the first M factors (a >= 2) take x^(a-1) from the power table
#pragma unroll
    for (int l = 0; l < M; ++l) pw[l] = ldsc(xb, h.po[l], lane);
    hnext = dfast_head<K, M>(rnext);
    // suffix products: sf[l] = x_l x_{l+1} ... x_{K-1}
    sf[K - 1] = xv[K - 1];
#pragma unroll
    for (int l = K - 2; l >= 1; --l) sf[l] = c_mul<1>(sf[l + 1], xv[l]);
    // common factor: c times the product of the M powers, as a balanced tree
    if constexpr (M > 0) {
#pragma unroll
        for (int st = 1; st < M; st *= 2) {
#pragma unroll
            for (int l = 0; l + st < M; l += 2 * st) pw[l] = c_mul<1>(pw[l], pw[l + st]);
        }
        cf = c_mul<1>(cf, pw[0]);
    }
    // q = c x_0 ... x_{l-1} (times the powers); partial l = q * sf[l+1],
    // scaled by the exponent a_l >= 2 for the first M factors; a factor with
    // exponent 1 has q * sf[l+1] accumulated straight into the row (four FMAs
    // in place of a product and two FMAs)
    C<1> q = cf;
#pragma unroll
    for (int l = 0; l < K - 1; ++l) {
        if (l >= M) {
            row.cfma((int)h.j2[l], q, sf[l + 1]);
        } else {
            const C<1> part = c_mul<1>(q, sf[l + 1]);
            row.fma((int)h.j2[l], h.a[l], part);
        }
        q = c_mul<1>(q, xv[l]);
    }
    v = c_add<1>(v, c_mul<1>(q, xv[K - 1]));
    row.fma((int)h.j2[K - 1], h.a[K - 1], q);
}

// All records of one equation, group by group: (K, M) = (1,0), (1,1), (2,0),
// ..., (8,8), each a straight-line loop over its records.
template <int K, int M, int KF, class Row>
__device__ __forceinline__ void dfast_groups(const int32_t *__restrict__ run, const DTerm *__restrict__ dterm,
                                             const char *__restrict__ xb, int lane, const C<1> &gs,
                                             double tv, Row &row, C<1> &v)
{
    constexpr int g = drun_group(K, M);
    const int s0 = run[g], s1 = run[g + 1];
    if (s0 < s1) {
        DHead h = dfast_head<K, M>(dterm + s0);
        for (int s = s0; s < s1; ++s) {
            const DTerm *rn = dterm + (s + 1 < s1 ? s + 1 : s);
            const C<1> c0 = c_from<1>(h.cre, h.cim);
            const C<1> c = (h.sel & 1) ? c_mul<1>(c0, gs) : c_mul_d<1>(c0, tv);
            DHead hn;
            dfast_sweep<K, M>(h, rn, hn, xb, lane, c, row, v);
            h = hn;
        }
    }
    if constexpr (M < K)
        dfast_groups<K, M + 1, KF>(run, dterm, xb, lane, gs, tv, row, v);
    else if constexpr (K < KF)
        dfast_groups<K + 1, 0, KF>(run, dterm, xb, lane, gs, tv, row, v);
}

// KF: largest number of factors per term the kernel handles; NC: largest
// number of unknowns (Jacobian columns held in the row).
template <class Row, int KF, int NC>
__device__ __forceinline__ void dfast_body(const EvalArgs &a, const int32_t *__restrict__ d_run,
                                           const DTerm *__restrict__ dterm,
                                           const int32_t *__restrict__ d_deg, int planes)
{
    extern __shared__ double xl[];
    const char *xb = reinterpret_cast<const char *>(xl);
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int W = blockDim.x >> 6;
    const int64_t p = (int64_t)blockIdx.x * 64 + lane;
    const bool act = p < a.npts;
    const int nv = a.n_var;
    // stage x and its powers: plane q holds x^(q+1)
    for (int var = w; var < nv; var += W) {
        C<1> x1 = act ? c_from<1>(a.x[(int64_t)(var * 2) * a.ld + p], a.x[(int64_t)(var * 2 + 1) * a.ld + p])
                      : c_zero<1>();
        C<1> z = x1;
        for (int q = 0; q < planes; ++q) {
            xl[((q * nv + var) * 2) * 64 + lane] = z.re.v[0];
            xl[((q * nv + var) * 2 + 1) * 64 + lane] = z.im.v[0];
            z = c_mul<1>(z, x1);
        }
    }
    if (w == 0) {
        xl[(planes * nv * 2) * 64 + lane] = 1.0;
        xl[(planes * nv * 2 + 1) * 64 + lane] = 0.0;
    }
    __syncthreads();

    double tv = 1.0;
    if (a.t) tv = act ? a.t[p] : 0.0;
    C<1> gs = c_zero<1>();
    if (a.t) gs = c_mul_d<1>(c_from<1>(a.gre, a.gim), 1.0 - tv);

    for (int i = blockIdx.y * W + w; i < a.n_eq; i += a.eq_stride) {
        Row row;
        row.zero();
        C<1> v = c_zero<1>();
        const int32_t *run = d_run + i * DRUN;
        auto coef = [&](const DTerm *r) -> C<1> {
            const C<1> c = c_from<1>(r->cre, r->cim);
            return (r->sel & 1) ? c_mul<1>(c, gs) : c_mul_d<1>(c, tv);
        };
        for (int s = run[0]; s < run[1]; ++s) v = c_add<1>(v, coef(dterm + s));
        dfast_groups<1, 0, KF>(run, dterm, xb, lane, gs, tv, row, v);
        // total-degree start part: gamma (1-t) (x_i^d - 1), derivative d x_i^(d-1)
        const int d = d_deg[i];
        if (d > 0 && a.t) {
            const C<1> xi = ldsc(xb, (uint32_t)(i * 2 * 64 * 8), lane);
            C<1> pw = c_from<1>(1.0, 0.0), base = xi;  // pw = x_i^(d-1)
            for (int e = d - 1; e > 0; e >>= 1) {
                if (e & 1) pw = c_mul<1>(pw, base);
                if (e > 1) base = c_mul<1>(base, base);
            }
            v = c_add<1>(v, c_mul<1>(gs, c_sub<1>(c_mul<1>(pw, xi), c_from<1>(1.0, 0.0))));
            row.fma(2 * i, (double)d, c_mul<1>(gs, pw));
        }
        if (act) {
            st_out(&a.val[((int64_t)(i * 2 + 0)) * a.ld + p], v.re.v[0]);
            st_out(&a.val[((int64_t)(i * 2 + 1)) * a.ld + p], v.im.v[0]);
            double *jr = a.jac + (int64_t)i * nv * 2 * a.ld + p;
            if constexpr (Row::kIndexed) {
                // a loop over the equation's own columns: the register index
                // is a loop counter, so no per-column bound or offset has to
                // be kept (an unrolled store kept 64 of them, spilled to
                // vector-register lanes and read back here)
                const int64_t ld2 = 2 * a.ld;
#pragma unroll 1
                for (int j = 0; j < nv; ++j, jr += ld2) {
                    double re, im;
                    row.get(j, re, im);
                    st_out(jr, re);
                    st_out(jr + a.ld, im);
                }
            } else {
#pragma unroll
                for (int j = 0; j < NC; ++j) {
                    if (j < nv) {
                        double re, im;
                        row.get(j, re, im);
                        st_out(&jr[(int64_t)(j * 2 + 0) * a.ld], re);
                        st_out(&jr[(int64_t)(j * 2 + 1) * a.ld], im);
                    }
                }
            }
        }
    }
}

__global__ void __launch_bounds__(512) eval_d_fast_kernel(EvalArgs a, const int32_t *__restrict__ d_run,
                                                          const DTerm *__restrict__ dterm,
                                                          const int32_t *__restrict__ d_deg, int planes)
{
    dfast_body<VecRow, 8, 32>(a, d_run, dterm, d_deg, planes);
}

// The same with the row pinned in v[128:255] (PinRow); everything else of
// the kernel lives in the lower 128 registers.
__global__ void __launch_bounds__(512) __attribute__((amdgpu_num_vgpr(128)))
eval_d_pinned_kernel(EvalArgs a, const int32_t *__restrict__ d_run, const DTerm *__restrict__ dterm,
                     const int32_t *__restrict__ d_deg, int planes)
{
    dfast_body<PinRow, 8, 32>(a, d_run, dterm, d_deg, planes);
}

// Systems with n <= 16 and at most two factors per term (PinRow16): four
// waves per SIMD for the evaluations that are bound by HBM traffic.
__global__ void __launch_bounds__(512) __attribute__((amdgpu_num_vgpr(64)))
eval_d_pinned16_kernel(EvalArgs a, const int32_t *__restrict__ d_run, const DTerm *__restrict__ dterm,
                       const int32_t *__restrict__ d_deg, int planes)
{
    dfast_body<PinRow16, 2, 16>(a, d_run, dterm, d_deg, planes);
}

template <int L, int KMAX, bool XLDS, bool JAC>
static int launch4(const EvalArgs &a, int W, int G, size_t lds, hipStream_t st)
{
    dim3 grid((unsigned)((a.npts + 63) / 64), (unsigned)G);
    if (L == 4 && W <= 4)
        hipLaunchKernelGGL((eval_kernel_w1<L, KMAX, XLDS, JAC>), grid, dim3(64 * W), XLDS ? lds : 0, st, a);
    else
        hipLaunchKernelGGL((eval_kernel<L, KMAX, XLDS, JAC>), grid, dim3(64 * W), XLDS ? lds : 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "eval_kernel launch");
    return PH_OK;
}

template <int L, int KMAX>
static int launch3(const EvalArgs &a, bool xlds, bool jac, int W, int G, size_t lds, hipStream_t st)
{
    if (xlds)
        return jac ? launch4<L, KMAX, true, true>(a, W, G, lds, st)
                   : launch4<L, KMAX, true, false>(a, W, G, lds, st);
    return jac ? launch4<L, KMAX, false, true>(a, W, G, lds, st)
               : launch4<L, KMAX, false, false>(a, W, G, lds, st);
}

template <int L>
static int launch2(const EvalArgs &a, int kmax, bool xlds, bool jac, int W, int G, size_t lds,
                   hipStream_t st)
{
    if (kmax <= 4) return launch3<L, 4>(a, xlds, jac, W, G, lds, st);
    if (kmax <= 8) return launch3<L, 8>(a, xlds, jac, W, G, lds, st);
    if (kmax <= 16) return launch3<L, 16>(a, xlds, jac, W, G, lds, st);
    return launch3<L, 32>(a, xlds, jac, W, G, lds, st);
}

int eval_launch(const DevTable &tab, const double gamma[2], int prec, int64_t npts,
                const double *t, const double *x, int64_t ld, double *val, double *jac,
                hipStream_t st, const EvalCfg *cfg)
{
    EvalArgs a;
    a.eq_off = tab.eq_off;
    a.tdesc = tab.tdesc;
    a.fac = tab.fac;
    a.coef = tab.coef;
    a.zc_off = tab.zc_off;
    a.zc = tab.zc;
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
    const bool wj = jac != nullptr;
    // which kernel: the fast path when its records exist, else the register
    // row in double, else the general kernel
    // fast path: double (register row), double double or quad double (row
    // in the accumulation registers)
    const bool can_fast = wj && tab.n_var <= 32 && tab.dfast && (prec == 1 || tab.mfast);
    const bool can_reg = prec == 1 && wj && tab.n_var <= 32 && tab.kmax <= 16;
    int kernel = cfg ? cfg->kernel : 0;
    if (kernel == 5) return unfused_launch(tab, gamma, prec, npts, t, x, ld, val, jac, st);
    // the register-row kernels produce the Jacobian; values alone take the
    // general kernel with the same tiling
    if (!wj && kernel >= 2) kernel = 1;
    if ((kernel == 3 || kernel == 4) && !can_fast)
        return fail(PH_EUNSUPPORTED, "fast path not available for this system");
    if (kernel == 4 && prec != 1)
        return fail(PH_EUNSUPPORTED, "the compiler-held row is a complex-double kernel");
    if (kernel == 2 && !can_reg) return fail(PH_EUNSUPPORTED, "register-row kernel not available");
    if (kernel == 0) kernel = can_fast ? 3 : (can_reg ? 2 : 1);
    if (kernel == 3 && prec == 2)
        return dd_fast_launch(tab, gamma, npts, t, x, ld, val, jac, cfg && cfg->W > 0 ? cfg->W : 4,
                              cfg && cfg->G > 0 ? cfg->G : 1, st);
    if (kernel == 3 && prec == 4)
        return qd_fast_launch(tab, gamma, npts, t, x, ld, val, jac, cfg && cfg->W > 0 ? cfg->W : 4,
                              cfg && cfg->G > 0 ? cfg->G : 1, st);
    if ((kernel == 3 || kernel == 4) && prec != 1)
        return fail(PH_EUNSUPPORTED, "fast path not available at this precision");
    // waves per workgroup: all of them share the 64 points staged in LDS and
    // take their own equations; wide precisions want more waves per
    // workgroup because their LDS tile (n * L KB) limits workgroups per CU
    // (a configured count is taken as it is, up to 8 and n_eq: six waves of
    // a 148-register kernel fill three waves per SIMD where eight cannot)
    int W = 1;
    if (cfg && cfg->W > 0) {
        W = cfg->W < 8 ? cfg->W : 8;
        if (W > tab.n_eq) W = tab.n_eq > 0 ? tab.n_eq : 1;
    } else {
        const int Wwant = kernel >= 2 ? 8 : (prec == 1 ? 4 : 8);
        while (W * 2 <= Wwant && W * 2 <= tab.n_eq && W * 2 <= 8) W *= 2;
    }
    const int64_t blocks = (npts + 63) / 64;
    int G = 1;
    if (cfg && cfg->G > 0) {
        while (G * 2 <= cfg->G && G * W * 2 <= tab.n_eq) G *= 2;
    } else {
        while (blocks * G < 1024 && G * W * 2 <= tab.n_eq) G *= 2;
    }
    a.eq_stride = G * W;
    dim3 grid((unsigned)blocks, (unsigned)G);
    const size_t lds = (size_t)tab.n_var * 2 * prec * 64 * sizeof(double);
    if (kernel == 3 || kernel == 4) {
        const size_t ldsf = ((size_t)tab.dfast_planes * tab.n_var * 2 + 2) * 64 * sizeof(double);
        if (kernel == 3 && tab.n_var <= 16 && tab.kmax <= 2)
            hipLaunchKernelGGL(eval_d_pinned16_kernel, grid, dim3(64 * W), ldsf, st, a, tab.d_run,
                               tab.dterm, tab.d_deg, tab.dfast_planes);
        else if (kernel == 3)
            hipLaunchKernelGGL(eval_d_pinned_kernel, grid, dim3(64 * W), ldsf, st, a, tab.d_run,
                               tab.dterm, tab.d_deg, tab.dfast_planes);
        else
            hipLaunchKernelGGL(eval_d_fast_kernel, grid, dim3(64 * W), ldsf, st, a, tab.d_run,
                               tab.dterm, tab.d_deg, tab.dfast_planes);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "fast-path kernel launch");
        return PH_OK;
    }
    if (kernel == 2) {
        if (tab.kmax <= 4)
            hipLaunchKernelGGL(eval_d_regrow_kernel<4>, grid, dim3(64 * W), lds, st, a);
        else if (tab.kmax <= 8)
            hipLaunchKernelGGL(eval_d_regrow_kernel<8>, grid, dim3(64 * W), lds, st, a);
        else
            hipLaunchKernelGGL(eval_d_regrow_kernel<16>, grid, dim3(64 * W), lds, st, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "eval_d_regrow_kernel launch");
        return PH_OK;
    }
    const bool xlds = lds <= 160 * 1024;
    switch (prec) {
    case 1: return launch2<1>(a, tab.kmax, xlds, wj, W, G, lds, st);
    case 2: return launch2<2>(a, tab.kmax, xlds, wj, W, G, lds, st);
    default: return launch2<4>(a, tab.kmax, xlds, wj, W, G, lds, st);
    }
}

static int eval_check(const ph_system *target, const ph_system *start, const double gamma[2],
                      int32_t prec, int64_t npts, const double *t, const double *x, int64_t ld,
                      const double *val)
{
    if (!target) return fail(PH_EINVAL, "null target system");
    if (prec != 1 && prec != 2 && prec != 4) return fail(PH_EINVAL, "prec must be 1, 2 or 4");
    if (npts < 0) return fail(PH_EINVAL, "npts < 0");
    if (npts == 0) return PH_OK;
    if (!x || !val) return fail(PH_EINVAL, "null x or val");
    if (ld < npts) return fail(PH_EINVAL, "ld < npts");
    if (start && (start->h.n_eq != target->h.n_eq || start->h.n_var != target->h.n_var))
        return fail(PH_EINVAL, "start system shape differs from target");
    if (!start && t && target->h.n_eq != target->h.n_var)
        return fail(PH_EINVAL, "the total-degree start system needs a square target");
    if (t && !gamma) return fail(PH_EINVAL, "gamma is null");
    return PH_OK;
}

// Look up a tuned configuration: in the handle, else among the entries of
// the PH_AUTOTUNE_CACHE file read when the target was created (memory only:
// an evaluation never touches the file system).
static bool eval_cfg_lookup(const ph_system *target, const ph_system *start, int prec, EvalCfg &out)
{
    ph_system *tg = const_cast<ph_system *>(target);
    std::lock_guard<std::mutex> lk(tg->mu);
    auto it = tg->eval_cfg.find({start, prec});
    if (it != tg->eval_cfg.end()) {
        out = it->second;
        return true;
    }
    auto ft = tg->file_cfg.find({start ? start->h.fingerprint : 0ull, prec});
    if (ft == tg->file_cfg.end()) return false;
    out = ft->second;
    tg->eval_cfg[{start, prec}] = out;
    return true;
}

}  // namespace ph

using namespace ph;

extern "C" int ph_eval_jac(const ph_system *target, const ph_system *start, const double gamma[2],
                           int32_t prec, int64_t npts, const double *t, const double *x, int64_t ld,
                           double *val, double *jac, void *stream)
{
    int rc = eval_check(target, start, gamma, prec, npts, t, x, ld, val);
    if (rc || npts == 0) return rc;
    const DevTable *tab = nullptr;
    rc = find_table(target, start, &tab);  // built by ph_system_create / ph_eval_prepare
    if (rc) return rc;
    EvalCfg cfg;
    const bool tuned = eval_cfg_lookup(target, start, prec, cfg);
    return eval_launch(*tab, gamma, prec, npts, t, x, ld, val, jac, (hipStream_t)stream,
                       tuned ? &cfg : nullptr);
}

extern "C" int ph_eval_prepare(ph_system *target, const ph_system *start, int32_t prec,
                               int64_t unfused_points)
{
    if (!target) return fail(PH_EINVAL, "null target system");
    if (prec != 1 && prec != 2 && prec != 4) return fail(PH_EINVAL, "prec must be 1, 2 or 4");
    if (unfused_points < 0) return fail(PH_EINVAL, "unfused_points < 0");
    if (start && (start->h.n_eq != target->h.n_eq || start->h.n_var != target->h.n_var))
        return fail(PH_EINVAL, "start system shape differs from target");
    const DevTable *tab = nullptr;
    int rc = get_table(target, start, &tab);
    if (rc) return rc;
    if (unfused_points > 0)
        rc = prepare_unfused(target, const_cast<DevTable &>(*tab), prec, unfused_points);
    return rc;
}

extern "C" int ph_eval_set_config(ph_system *target, const ph_system *start, int32_t prec,
                                  int32_t kernel, int32_t waves, int32_t groups)
{
    if (!target) return fail(PH_EINVAL, "null target system");
    if (prec != 1 && prec != 2 && prec != 4) return fail(PH_EINVAL, "prec must be 1, 2 or 4");
    if (kernel < 0 || kernel > 5 || waves < 0 || waves > 8 || groups < 0)
        return fail(PH_EINVAL, "kernel must be 0..5, waves 0..8, groups >= 0");
    std::lock_guard<std::mutex> lk(target->mu);
    if (kernel == 0 && waves == 0 && groups == 0)
        target->eval_cfg.erase({start, prec});
    else
        target->eval_cfg[{start, prec}] = EvalCfg{kernel, waves, groups};
    return PH_OK;
}

extern "C" int ph_eval_get_config(const ph_system *target, const ph_system *start, int32_t prec,
                                  int32_t *kernel, int32_t *waves, int32_t *groups)
{
    if (!target || !kernel || !waves || !groups) return fail(PH_EINVAL, "null argument");
    // the same lookup ph_eval_jac makes: the handle, else the cache file
    EvalCfg c{0, 0, 0};
    if (!eval_cfg_lookup(target, start, prec, c)) c = EvalCfg{0, 0, 0};
    *kernel = c.kernel;
    *waves = c.W;
    *groups = c.G;
    return PH_OK;
}

extern "C" int ph_eval_autotune(ph_system *target, const ph_system *start, const double gamma[2],
                                int32_t prec, int64_t npts, const double *t, const double *x,
                                int64_t ld, double *val, double *jac, void *stream,
                                double *best_ms)
{
    int rc = eval_check(target, start, gamma, prec, npts, t, x, ld, val);
    if (rc) return rc;
    if (npts == 0) return fail(PH_EINVAL, "autotuning needs npts > 0");
    const DevTable *tab = nullptr;
    rc = get_table(target, start, &tab);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    PH_HIP(hipEventCreate(&e0));
    PH_HIP(hipEventCreate(&e1));
    EvalCfg best;
    double best_t = 1e300;
    const int kernels[4] = {3, 4, 2, 1};
    for (int kk : kernels) {
        for (int W : {1, 2, 4, 6, 8}) {
            for (int G = 1; G <= 8; G *= 2) {
                if (W * G > tab->n_eq) continue;
                EvalCfg c{kk, W, G};
                rc = eval_launch(*tab, gamma, prec, npts, t, x, ld, val, jac, st, &c);
                if (rc == PH_EUNSUPPORTED) break;  // this kernel does not apply
                if (rc) goto done;
                (void)hipEventRecord(e0, st);
                for (int r = 0; r < 3 && !rc; ++r) rc = eval_launch(*tab, gamma, prec, npts, t, x, ld, val, jac, st, &c);
                (void)hipEventRecord(e1, st);
                if (rc) goto done;
                if (hipEventSynchronize(e1) != hipSuccess) {
                    rc = fail(PH_EHIP, "autotune timing");
                    goto done;
                }
                float ms = 0;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (ms / 3.0 < best_t) {
                    best_t = ms / 3.0;
                    best = c;
                }
            }
            if (rc == PH_EUNSUPPORTED) break;
        }
        rc = PH_OK;
    }
    {
        std::lock_guard<std::mutex> lk(target->mu);
        target->eval_cfg[{start, prec}] = best;
    }
    if (const char *path = std::getenv("PH_AUTOTUNE_CACHE")) {
        if (FILE *f = std::fopen(path, "a")) {
            std::fprintf(f, "eval %llx %llx %d %d %d %d %.6f\n", (unsigned long long)target->h.fingerprint,
                         (unsigned long long)(start ? start->h.fingerprint : 0ull), prec, best.kernel,
                         best.W, best.G, best_t);
            std::fclose(f);
        }
    }
    if (best_ms) *best_ms = best_t;
done:
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}
