// ph_arith.hpp -- complex double, double double and quad double arithmetic for
// gfx950, the three precisions of the paper (Section 1: DD and QD make the
// evaluation compute bound).  Written from the published error-free
// transformations:
//   * TwoSum (Knuth): s + e = a + b exactly, 6 FP64 operations;
//   * FastTwoSum (Dekker): the same in 3 operations when |a| >= |b| or a = 0;
//   * TwoProd with a fused multiply-add: p + e = a * b exactly, 2 operations.
// A DD number is hi + lo with |lo| <= ulp(hi)/2 (roughly); a QD number is four
// such limbs.  DD addition is the accurate two-TwoSum form; DD multiplication
// adds the cross products into the FMA error term (Joldes-Muller-Popescu,
// "Tight and rigorous error bounds for basic building blocks of double-word
// arithmetic", 2017, bounds of a few u^2).  QD follows the level-by-level
// scheme of Hida, Li and Bailey ("Algorithms for quad-double precision
// floating point arithmetic", 2001): partial products / sums are grouped by
// their order of magnitude (eps^0, eps^1, ...), each level is summed with
// TwoSum chains whose errors flow to the next level, and the result is
// renormalised; terms below eps^4 are dropped.  Relative error per operation
// stays near 2^-205, far below the parity bar (1e-52 ~ 2^-172).
//
// Compile with -ffp-contract=off: every FMA below is explicit and every other
// operation must round separately for the transformations to be exact.
#pragma once

#include <hip/hip_runtime.h>

#define PH_HD __host__ __device__ __forceinline__

namespace ph {

PH_HD void two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

PH_HD void fast_two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    e = b - (s - a);
}

PH_HD void two_prod(double a, double b, double &p, double &e)
{
    p = a * b;
    e = __builtin_fma(a, b, -p);
}

// ---------------------------------------------------------------------------
// L-limb reals
// ---------------------------------------------------------------------------
template <int L>
struct R {
    double v[L];
};

template <int L>
PH_HD R<L> r_zero()
{
    R<L> r;
#pragma unroll
    for (int l = 0; l < L; ++l) r.v[l] = 0.0;
    return r;
}

template <int L>
PH_HD R<L> r_from(double a)
{
    R<L> r = r_zero<L>();
    r.v[0] = a;
    return r;
}

template <int L>
PH_HD R<L> r_neg(R<L> a)
{
#pragma unroll
    for (int l = 0; l < L; ++l) a.v[l] = -a.v[l];
    return a;
}

// Renormalise five level-ordered components (c0 of order 1, c_k of order
// eps^k) into four limbs.  Pass 1 runs FastTwoSum from the bottom up, which
// leaves c0 = the rounded total and every c_k a rounding error no larger than
// half an ulp of the partial sum above it; pass 2 runs TwoSum over c1..c4
// from the bottom up, which closes any gap (a tiny c1 above a larger c2) so
// that |c_{k+1}| <= ulp(c_k).  The last component is folded in rounded.
PH_HD R<4> qd_renorm(double c0, double c1, double c2, double c3, double c4)
{
    double s;
    fast_two_sum(c3, c4, s, c4);
    fast_two_sum(c2, s, s, c3);
    fast_two_sum(c1, s, s, c2);
    fast_two_sum(c0, s, c0, c1);
    two_sum(c3, c4, s, c4);
    two_sum(c2, s, s, c3);
    two_sum(c1, s, c1, c2);
    c3 += c4;
    R<4> r;
    r.v[0] = c0;
    r.v[1] = c1;
    r.v[2] = c2;
    r.v[3] = c3;
    return r;
}

// The same when cancellation may have left a leading component smaller than a
// trailing one (after a subtraction): TwoSum in both passes.
PH_HD R<4> qd_renorm_safe(double c0, double c1, double c2, double c3, double c4)
{
    double s;
    two_sum(c3, c4, s, c4);
    two_sum(c2, s, s, c3);
    two_sum(c1, s, s, c2);
    two_sum(c0, s, c0, c1);
    two_sum(c3, c4, s, c4);
    two_sum(c2, s, s, c3);
    two_sum(c1, s, c1, c2);
    c3 += c4;
    R<4> r;
    r.v[0] = c0;
    r.v[1] = c1;
    r.v[2] = c2;
    r.v[3] = c3;
    return r;
}

template <int L>
PH_HD R<L> r_add(R<L> a, R<L> b)
{
    if constexpr (L == 1) {
        return R<1>{{a.v[0] + b.v[0]}};
    } else if constexpr (L == 2) {
        double s, e, t, f;
        two_sum(a.v[0], b.v[0], s, e);
        two_sum(a.v[1], b.v[1], t, f);
        e += t;
        fast_two_sum(s, e, s, e);
        e += f;
        fast_two_sum(s, e, s, e);
        return R<2>{{s, e}};
    } else {
        // level 0..3 pairwise sums; errors flow one level down
        double s0, e0, s1, e1, s2, e2, s3, e3;
        two_sum(a.v[0], b.v[0], s0, e0);
        two_sum(a.v[1], b.v[1], s1, e1);
        two_sum(a.v[2], b.v[2], s2, e2);
        two_sum(a.v[3], b.v[3], s3, e3);
        double u, w;
        two_sum(s1, e0, s1, u);      // level 1; u -> level 2
        two_sum(s2, e1, s2, w);      // level 2; w -> level 3
        two_sum(s2, u, s2, u);       // u -> level 3
        double x;
        two_sum(s3, e2, s3, x);      // level 3; x -> level 4
        two_sum(s3, w, s3, w);
        two_sum(s3, u, s3, u);
        double c4 = e3 + x + w + u;  // level 4 (only its leading bits survive)
        return qd_renorm_safe(s0, s1, s2, s3, c4);
    }
}

template <int L>
PH_HD R<L> r_sub(R<L> a, R<L> b)
{
    return r_add<L>(a, r_neg<L>(b));
}

template <int L>
PH_HD R<L> r_mul(R<L> a, R<L> b)
{
    if constexpr (L == 1) {
        return R<1>{{a.v[0] * b.v[0]}};
    } else if constexpr (L == 2) {
        double p, e;
        two_prod(a.v[0], b.v[0], p, e);
        e = __builtin_fma(a.v[0], b.v[1], e);
        e = __builtin_fma(a.v[1], b.v[0], e);
        fast_two_sum(p, e, p, e);
        return R<2>{{p, e}};
    } else {
        double p00, q00, p01, q01, p10, q10, p02, q02, p11, q11, p20, q20;
        two_prod(a.v[0], b.v[0], p00, q00);
        two_prod(a.v[0], b.v[1], p01, q01);
        two_prod(a.v[1], b.v[0], p10, q10);
        two_prod(a.v[0], b.v[2], p02, q02);
        two_prod(a.v[1], b.v[1], p11, q11);
        two_prod(a.v[2], b.v[0], p20, q20);
        // level 3: products of order eps^3 (rounded) and the level-2 errors
        double c3 = __builtin_fma(a.v[0], b.v[3], a.v[1] * b.v[2]);
        c3 = __builtin_fma(a.v[2], b.v[1], c3);
        c3 = __builtin_fma(a.v[3], b.v[0], c3);
        c3 += q02 + q11 + q20;
        // level 1: p01 + p10 + q00
        double c1, u1, u2;
        two_sum(p01, p10, c1, u1);
        two_sum(c1, q00, c1, u2);
        // level 2: p02 + p11 + p20 + q01 + q10 + u1 + u2
        double c2, w0, w1, w2, w3, w4, w5;
        two_sum(p02, p11, c2, w0);
        two_sum(c2, p20, c2, w1);
        two_sum(c2, q01, c2, w2);
        two_sum(c2, q10, c2, w3);
        two_sum(c2, u1, c2, w4);
        two_sum(c2, u2, c2, w5);
        c3 += ((w0 + w1) + (w2 + w3)) + (w4 + w5);
        return qd_renorm(p00, c1, c2, c3, 0.0);
    }
}

// a * b with b a double
template <int L>
PH_HD R<L> r_mul_d(R<L> a, double b)
{
    if constexpr (L == 1) {
        return R<1>{{a.v[0] * b}};
    } else if constexpr (L == 2) {
        double p, e;
        two_prod(a.v[0], b, p, e);
        e = __builtin_fma(a.v[1], b, e);
        fast_two_sum(p, e, p, e);
        return R<2>{{p, e}};
    } else {
        double p0, q0, p1, q1, p2, q2;
        two_prod(a.v[0], b, p0, q0);
        two_prod(a.v[1], b, p1, q1);
        two_prod(a.v[2], b, p2, q2);
        double c3 = __builtin_fma(a.v[3], b, q2);
        double c1, u, c2, w0, w1;
        two_sum(p1, q0, c1, u);
        two_sum(p2, q1, c2, w0);
        two_sum(c2, u, c2, w1);
        c3 += w0 + w1;
        return qd_renorm(p0, c1, c2, c3, 0.0);
    }
}

// a * b + c * d in quad double with one renormalisation (the complex
// product's components): the partial products of both pairs are grouped by
// order of magnitude as in r_mul<4>, the levels 0..2 are summed with TwoSum
// chains whose errors flow one level down, level 3 (products of order eps^3
// and the level-2 errors) is summed in plain FP64, and the result is
// renormalised once with TwoSum in both passes (a * b + c * d may cancel).
// Error a few 2^-210 times |a b| + |c d|.
PH_HD R<4> qd_dot2(const R<4> &a, const R<4> &b, const R<4> &c, const R<4> &d)
{
    // level 0
    double p0, e00, r0, f00, s0, t0;
    two_prod(a.v[0], b.v[0], p0, e00);
    two_prod(c.v[0], d.v[0], r0, f00);
    two_sum(p0, r0, s0, t0);
    // level 1: a0 b1, a1 b0, c0 d1, c1 d0, the two level-0 product errors, t0
    double p1a, e01, p1b, e10, r1a, f01, r1b, f10;
    two_prod(a.v[0], b.v[1], p1a, e01);
    two_prod(a.v[1], b.v[0], p1b, e10);
    two_prod(c.v[0], d.v[1], r1a, f01);
    two_prod(c.v[1], d.v[0], r1b, f10);
    double s1, u1, u2, u3, u4, u5, u6;
    two_sum(p1a, p1b, s1, u1);
    two_sum(s1, r1a, s1, u2);
    two_sum(s1, r1b, s1, u3);
    two_sum(s1, e00, s1, u4);
    two_sum(s1, f00, s1, u5);
    two_sum(s1, t0, s1, u6);
    // level 2: the six products of order eps^2 and the level-1 errors
    double p2a, e02, p2b, e11, p2c, e20, r2a, f02, r2b, f11, r2c, f20;
    two_prod(a.v[0], b.v[2], p2a, e02);
    two_prod(a.v[1], b.v[1], p2b, e11);
    two_prod(a.v[2], b.v[0], p2c, e20);
    two_prod(c.v[0], d.v[2], r2a, f02);
    two_prod(c.v[1], d.v[1], r2b, f11);
    two_prod(c.v[2], d.v[0], r2c, f20);
    double s2, w[15];
    two_sum(p2a, p2b, s2, w[0]);
    two_sum(s2, p2c, s2, w[1]);
    two_sum(s2, r2a, s2, w[2]);
    two_sum(s2, r2b, s2, w[3]);
    two_sum(s2, r2c, s2, w[4]);
    two_sum(s2, e01, s2, w[5]);
    two_sum(s2, e10, s2, w[6]);
    two_sum(s2, f01, s2, w[7]);
    two_sum(s2, f10, s2, w[8]);
    two_sum(s2, u1, s2, w[9]);
    two_sum(s2, u2, s2, w[10]);
    two_sum(s2, u3, s2, w[11]);
    two_sum(s2, u4, s2, w[12]);
    two_sum(s2, u5, s2, w[13]);
    two_sum(s2, u6, s2, w[14]);
    // level 3: products of order eps^3 (rounded), the level-2 product
    // errors and the level-2 sum errors
    double s3 = __builtin_fma(a.v[0], b.v[3], a.v[1] * b.v[2]);
    s3 = __builtin_fma(a.v[2], b.v[1], s3);
    s3 = __builtin_fma(a.v[3], b.v[0], s3);
    s3 = __builtin_fma(c.v[0], d.v[3], s3);
    s3 = __builtin_fma(c.v[1], d.v[2], s3);
    s3 = __builtin_fma(c.v[2], d.v[1], s3);
    s3 = __builtin_fma(c.v[3], d.v[0], s3);
    s3 += ((e02 + e11) + (e20 + f02)) + ((f11 + f20) + (w[0] + w[1]));
    s3 += ((w[2] + w[3]) + (w[4] + w[5])) + ((w[6] + w[7]) + (w[8] + w[9]));
    s3 += ((w[10] + w[11]) + (w[12] + w[13])) + w[14];
    return qd_renorm_safe(s0, s1, s2, s3, 0.0);
}

// ---------------------------------------------------------------------------
// L-limb complex numbers
// ---------------------------------------------------------------------------
template <int L>
struct C {
    R<L> re, im;
};

template <int L>
PH_HD C<L> c_zero()
{
    return C<L>{r_zero<L>(), r_zero<L>()};
}

template <int L>
PH_HD C<L> c_from(double re, double im)
{
    return C<L>{r_from<L>(re), r_from<L>(im)};
}

template <int L>
PH_HD C<L> c_add(C<L> a, C<L> b)
{
    return C<L>{r_add<L>(a.re, b.re), r_add<L>(a.im, b.im)};
}

template <int L>
PH_HD C<L> c_sub(C<L> a, C<L> b)
{
    return C<L>{r_sub<L>(a.re, b.re), r_sub<L>(a.im, b.im)};
}

// Complex product.  Double: four FMA-style operations.  Double double: each
// component a*b - c*d is formed from the two leading exact products (TwoProd)
// combined by one TwoSum, the four cross terms and the two product errors
// folded into the error term, then one FastTwoSum.  Quad double: each
// component a*b +- c*d by qd_dot2 (one renormalisation per component).
template <int L>
PH_HD C<L> c_mul(C<L> a, C<L> b)
{
    if constexpr (L == 1) {
        double re = __builtin_fma(a.re.v[0], b.re.v[0], -(a.im.v[0] * b.im.v[0]));
        double im = __builtin_fma(a.re.v[0], b.im.v[0], a.im.v[0] * b.re.v[0]);
        return C<1>{{{re}}, {{im}}};
    } else if constexpr (L == 2) {
        C<2> r;
        {
            double p1, e1, p2, e2, s, e;
            two_prod(a.re.v[0], b.re.v[0], p1, e1);
            two_prod(a.im.v[0], b.im.v[0], p2, e2);
            two_sum(p1, -p2, s, e);
            e += e1 - e2;
            e = __builtin_fma(a.re.v[0], b.re.v[1], e);
            e = __builtin_fma(a.re.v[1], b.re.v[0], e);
            e = __builtin_fma(-a.im.v[0], b.im.v[1], e);
            e = __builtin_fma(-a.im.v[1], b.im.v[0], e);
            fast_two_sum(s, e, r.re.v[0], r.re.v[1]);
        }
        {
            double p1, e1, p2, e2, s, e;
            two_prod(a.re.v[0], b.im.v[0], p1, e1);
            two_prod(a.im.v[0], b.re.v[0], p2, e2);
            two_sum(p1, p2, s, e);
            e += e1 + e2;
            e = __builtin_fma(a.re.v[0], b.im.v[1], e);
            e = __builtin_fma(a.re.v[1], b.im.v[0], e);
            e = __builtin_fma(a.im.v[0], b.re.v[1], e);
            e = __builtin_fma(a.im.v[1], b.re.v[0], e);
            fast_two_sum(s, e, r.im.v[0], r.im.v[1]);
        }
        return r;
    } else {
        return C<4>{qd_dot2(a.re, b.re, r_neg<4>(a.im), b.im), qd_dot2(a.re, b.im, a.im, b.re)};
    }
}

// complex times real L-limb
template <int L>
PH_HD C<L> c_mul_r(C<L> a, R<L> s)
{
    return C<L>{r_mul<L>(a.re, s), r_mul<L>(a.im, s)};
}

// complex times a double (exact scalings by small integers included)
template <int L>
PH_HD C<L> c_mul_d(C<L> a, double s)
{
    return C<L>{r_mul_d<L>(a.re, s), r_mul_d<L>(a.im, s)};
}

// L-limb complex times an FP64 complex (coefficients of a system are FP64)
template <int L>
PH_HD C<L> c_mul_c64(C<L> a, double br, double bi)
{
    if constexpr (L == 1) {
        double re = __builtin_fma(a.re.v[0], br, -(a.im.v[0] * bi));
        double im = __builtin_fma(a.re.v[0], bi, a.im.v[0] * br);
        return C<1>{{{re}}, {{im}}};
    } else {
        return C<L>{r_sub<L>(r_mul_d<L>(a.re, br), r_mul_d<L>(a.im, bi)),
                    r_add<L>(r_mul_d<L>(a.re, bi), r_mul_d<L>(a.im, br))};
    }
}

// 1/b by Newton's iteration y <- y + y (1 - b y) from the FP64 reciprocal of
// the leading limb; every step doubles the correct bits (53 -> 106 -> 212).
template <int L>
PH_HD R<L> r_recip(R<L> b)
{
    R<L> y = r_from<L>(1.0 / b.v[0]);
    if constexpr (L > 1) {
        const int steps = L == 2 ? 1 : 2;
        for (int s = 0; s < steps; ++s) {
            R<L> e = r_sub<L>(r_from<L>(1.0), r_mul<L>(b, y));
            y = r_add<L>(y, r_mul<L>(y, e));
        }
    }
    return y;
}

// a / b = a (1/b) plus one correction term y (a - b q).
template <int L>
PH_HD R<L> r_div(R<L> a, R<L> b)
{
    if constexpr (L == 1) {
        return R<1>{{a.v[0] / b.v[0]}};
    } else {
        R<L> y = r_recip<L>(b);
        R<L> q = r_mul<L>(a, y);
        R<L> e = r_sub<L>(a, r_mul<L>(b, q));
        return r_add<L>(q, r_mul<L>(y, e));
    }
}

// sqrt(a), a >= 0: 1/sqrt(a) by Newton y <- y + y (1 - a y^2) / 2 from the
// FP64 seed, then s = a y corrected once by s + y (a - s^2) / 2.
template <int L>
PH_HD R<L> r_sqrt(R<L> a)
{
    if (!(a.v[0] > 0.0)) return r_zero<L>();
    if constexpr (L == 1) {
        return R<1>{{sqrt(a.v[0])}};
    } else {
        R<L> y = r_from<L>(1.0 / sqrt(a.v[0]));
        const int steps = L == 2 ? 1 : 2;
        for (int s = 0; s < steps; ++s) {
            R<L> e = r_sub<L>(r_from<L>(1.0), r_mul<L>(a, r_mul<L>(y, y)));
            y = r_add<L>(y, r_mul_d<L>(r_mul<L>(y, e), 0.5));
        }
        R<L> sq = r_mul<L>(a, y);
        R<L> e = r_sub<L>(a, r_mul<L>(sq, sq));
        return r_add<L>(sq, r_mul_d<L>(r_mul<L>(y, e), 0.5));
    }
}

// conj(a) * b
template <int L>
PH_HD C<L> c_cmul(C<L> a, C<L> b)
{
    a.im = r_neg<L>(a.im);
    return c_mul<L>(a, b);
}

// |a|^2 as an L-limb real
template <int L>
PH_HD R<L> c_abs2(C<L> a)
{
    return r_add<L>(r_mul<L>(a.re, a.re), r_mul<L>(a.im, a.im));
}

// a + b with b an FP64 complex (the mixed-precision Newton update)
template <int L>
PH_HD C<L> c_add_c64(C<L> a, double br, double bi)
{
    C<L> b = c_from<L>(br, bi);
    return c_add<L>(a, b);
}

// Generic names used by the term sweep.
template <int L>
PH_HD C<L> num_mul(C<L> a, C<L> b)
{
    return c_mul<L>(a, b);
}

template <int L>
PH_HD C<L> num_scale(C<L> a, double s)
{
    return c_mul_d<L>(a, s);
}

// Leading limb (the FP64 value handed to the FP64 corrector).
template <int L>
PH_HD double r_hi(R<L> a)
{
    return a.v[0];
}

} // namespace ph
