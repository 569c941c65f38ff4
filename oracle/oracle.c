/*
 * oracle.c -- slow, plain CPU oracle for the many-path homotopy hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The product path
 * (the HIP library and its binding) never calls it, and the two share no code.
 *
 * What it computes (each function names the passage of Verschelde & Yu,
 * "Tracking Many Solution Paths of a Polynomial Homotopy on a GPU", 2015):
 *
 *   - multi-limb real/complex arithmetic with L = 1, 2 or 4 limbs (double,
 *     double double, quad double; Section 1 motivates the three precisions).
 *     Every operation is computed EXACTLY as a floating-point expansion
 *     (Knuth's TwoSum, Dekker's TwoProduct with Veltkamp splitting -- no fused
 *     multiply-add anywhere -- and Shewchuk's Grow-Expansion), then cut to its
 *     L limbs by taking the floating-point value of the exact remainder limb
 *     after limb.  Division and square root are Newton
 *     iterations seeded in FP64.
 *   - evaluation of the homotopy gamma(1-t)g(x) + t f(x) (Eq. (1)) and its
 *     Jacobian at one point, following the host pseudo code of Table 4: per
 *     polynomial, per monomial, coefficient times monomial and the symbolic
 *     derivative of the monomial computed DIRECTLY (no reverse mode, no reuse
 *     of partial products), added into the values and the Jacobian.
 *   - least squares by modified Gram-Schmidt (Section 1: Newton's linear
 *     systems are solved in the least squares sense by MGS; Section 3, QR in
 *     the corrector).
 *   - the path tracker of Section 2 (Tables 1-3): predict, evaluate-correct
 *     until converged, per-path t and step size, status 0 / -1 / 1, followed
 *     by a Newton polish at t = 1.
 *
 * Compile with -O2 -ffp-contract=off and never with -ffast-math: the
 * error-free transformations below rely on every operation being rounded
 * separately.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MAXL 4
#define EXPCAP 160

/* ------------------------------------------------------------------------ */
/* Error-free transformations                                                */
/* ------------------------------------------------------------------------ */

/* Knuth's TwoSum: s + e == a + b exactly, s = fl(a + b). */
static void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double bv = x - a;
    double av = x - bv;
    double br = b - bv;
    double ar = a - av;
    *s = x;
    *e = ar + br;
}

/* Veltkamp's splitting of a double into two halves of at most 26 bits. */
static void split(double a, double *hi, double *lo)
{
    const double c = 134217729.0; /* 2^27 + 1 */
    double t = c * a;
    double ab = t - a;
    *hi = t - ab;
    *lo = a - *hi;
}

/* Dekker's TwoProduct without FMA: p + e == a * b exactly, p = fl(a * b). */
static void two_prod(double a, double b, double *p, double *e)
{
    double x = a * b;
    double ah, al, bh, bl;
    split(a, &ah, &al);
    split(b, &bh, &bl);
    double e1 = x - ah * bh;
    double e2 = e1 - al * bh;
    double e3 = e2 - ah * bl;
    *p = x;
    *e = al * bl - e3;
}

/* ------------------------------------------------------------------------ */
/* Expansions: arrays of doubles, non-overlapping, increasing magnitude,     */
/* zero components removed.  The represented value is the exact sum.        */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n;
    double c[EXPCAP];
} expn;

static void ex_zero(expn *e) { e->n = 0; }

/* Shewchuk's Grow-Expansion with zero elimination: e <- e + b exactly. */
static void ex_add_d(expn *e, double b)
{
    double q = b;
    int m = 0;
    for (int i = 0; i < e->n; ++i) {
        double s, h;
        two_sum(q, e->c[i], &s, &h);
        q = s;
        if (h != 0.0) e->c[m++] = h;
    }
    if (q != 0.0) {
        if (m >= EXPCAP) abort();
        e->c[m++] = q;
    }
    e->n = m;
}

/* e <- e + a * b exactly (TwoProduct, then two Grow steps). */
static void ex_add_prod(expn *e, double a, double b)
{
    double p, q;
    two_prod(a, b, &p, &q);
    ex_add_d(e, q);
    ex_add_d(e, p);
}

/* Floating-point sum of an expansion, smallest component first.  Because the
 * components are non-overlapping and increasing, the result is within a few
 * ulps of the exact value. */
static double ex_approx(const expn *e)
{
    double s = 0.0;
    for (int i = 0; i < e->n; ++i) s += e->c[i];
    return s;
}

/* Cut an expansion to L limbs: limb l is the floating-point sum of what is
 * left, which is then subtracted exactly.  What remains after L limbs is a few
 * ulps of the last limb, so the L-limb value has relative error ~2^(-52 L). */
static void ex_round(const expn *e, int L, double *out)
{
    expn r = *e;
    for (int l = 0; l < L; ++l) {
        double v = ex_approx(&r);
        out[l] = v;
        if (v != 0.0) ex_add_d(&r, -v);
    }
}

/* ------------------------------------------------------------------------ */
/* L-limb reals: double[MAXL], value = sum of the first L entries.           */
/* ------------------------------------------------------------------------ */
typedef struct {
    double v[MAXL];
} mp;

static mp mp_d(double a)
{
    mp r;
    memset(&r, 0, sizeof r);
    r.v[0] = a;
    return r;
}

static void ex_add_mp(expn *e, int L, const mp *a, double sign)
{
    for (int l = L - 1; l >= 0; --l) ex_add_d(e, sign * a->v[l]);
}

static void ex_add_mpprod(expn *e, int L, const mp *a, const mp *b, double sign)
{
    for (int i = L - 1; i >= 0; --i)
        for (int j = L - 1; j >= 0; --j) ex_add_prod(e, sign * a->v[i], b->v[j]);
}

static mp ex_to_mp(const expn *e, int L)
{
    mp r;
    memset(&r, 0, sizeof r);
    ex_round(e, L, r.v);
    return r;
}

static mp mp_add(int L, mp a, mp b)
{
    expn e;
    ex_zero(&e);
    ex_add_mp(&e, L, &a, 1.0);
    ex_add_mp(&e, L, &b, 1.0);
    return ex_to_mp(&e, L);
}

static mp mp_sub(int L, mp a, mp b)
{
    expn e;
    ex_zero(&e);
    ex_add_mp(&e, L, &a, 1.0);
    ex_add_mp(&e, L, &b, -1.0);
    return ex_to_mp(&e, L);
}

static mp mp_mul(int L, mp a, mp b)
{
    expn e;
    ex_zero(&e);
    ex_add_mpprod(&e, L, &a, &b, 1.0);
    return ex_to_mp(&e, L);
}

static mp mp_neg(int L, mp a)
{
    for (int l = 0; l < L; ++l) a.v[l] = -a.v[l];
    return a;
}

static double mp_hi(mp a) { return a.v[0]; }

/* 1/b by Newton's iteration y <- y + y(1 - b y), seeded with 1/b_hi in FP64.
 * Each step doubles the number of correct bits: 53 -> 106 -> 212 -> 424. */
static mp mp_recip(int L, mp b)
{
    mp y = mp_d(1.0 / b.v[0]);
    int steps = L == 1 ? 0 : (L == 2 ? 2 : 3);
    for (int s = 0; s < steps; ++s) {
        mp r = mp_sub(L, mp_d(1.0), mp_mul(L, b, y));
        y = mp_add(L, y, mp_mul(L, y, r));
    }
    return y;
}

/* a / b: q = a * (1/b), then one correction q + y (a - b q). */
static mp mp_div(int L, mp a, mp b)
{
    if (L == 1) return mp_d(a.v[0] / b.v[0]);
    mp y = mp_recip(L, b);
    mp q = mp_mul(L, a, y);
    mp r = mp_sub(L, a, mp_mul(L, b, q));
    return mp_add(L, q, mp_mul(L, y, r));
}

/* sqrt(a) for a >= 0: 1/sqrt(a) by Newton y <- y + y (1 - a y^2)/2, then
 * s = a y corrected once by s + y (a - s^2)/2. */
static mp mp_sqrt(int L, mp a)
{
    if (a.v[0] <= 0.0) return mp_d(0.0);
    if (L == 1) return mp_d(sqrt(a.v[0]));
    mp y = mp_d(1.0 / sqrt(a.v[0]));
    int steps = L == 2 ? 2 : 3;
    for (int s = 0; s < steps; ++s) {
        mp r = mp_sub(L, mp_d(1.0), mp_mul(L, a, mp_mul(L, y, y)));
        mp hr = r;
        for (int l = 0; l < L; ++l) hr.v[l] *= 0.5; /* exact */
        y = mp_add(L, y, mp_mul(L, y, hr));
    }
    mp s = mp_mul(L, a, y);
    mp r = mp_sub(L, a, mp_mul(L, s, s));
    for (int l = 0; l < L; ++l) r.v[l] *= 0.5;
    return mp_add(L, s, mp_mul(L, y, r));
}

/* ------------------------------------------------------------------------ */
/* L-limb complex numbers.  Each component of a product is formed exactly   */
/* as an expansion and cut to L limbs once.                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    mp re, im;
} cx;

static cx cx_zero(void)
{
    cx z;
    memset(&z, 0, sizeof z);
    return z;
}

static cx cx_d(double re, double im)
{
    cx z = cx_zero();
    z.re.v[0] = re;
    z.im.v[0] = im;
    return z;
}

static cx cx_add(int L, cx a, cx b)
{
    cx r;
    r.re = mp_add(L, a.re, b.re);
    r.im = mp_add(L, a.im, b.im);
    return r;
}

static cx cx_sub(int L, cx a, cx b)
{
    cx r;
    r.re = mp_sub(L, a.re, b.re);
    r.im = mp_sub(L, a.im, b.im);
    return r;
}

static cx cx_mul(int L, cx a, cx b)
{
    expn e;
    cx r;
    ex_zero(&e);
    ex_add_mpprod(&e, L, &a.re, &b.re, 1.0);
    ex_add_mpprod(&e, L, &a.im, &b.im, -1.0);
    r.re = ex_to_mp(&e, L);
    ex_zero(&e);
    ex_add_mpprod(&e, L, &a.re, &b.im, 1.0);
    ex_add_mpprod(&e, L, &a.im, &b.re, 1.0);
    r.im = ex_to_mp(&e, L);
    return r;
}

/* conj(a) * b */
static cx cx_cmul(int L, cx a, cx b)
{
    a.im = mp_neg(L, a.im);
    return cx_mul(L, a, b);
}

static cx cx_scale(int L, cx a, mp s)
{
    cx r;
    r.re = mp_mul(L, a.re, s);
    r.im = mp_mul(L, a.im, s);
    return r;
}

/* |a|^2 as an L-limb real, formed exactly then cut. */
static mp cx_abs2(int L, cx a)
{
    expn e;
    ex_zero(&e);
    ex_add_mpprod(&e, L, &a.re, &a.re, 1.0);
    ex_add_mpprod(&e, L, &a.im, &a.im, 1.0);
    return ex_to_mp(&e, L);
}

static double cx_absd(cx a) { return hypot(a.re.v[0], a.im.v[0]); }

/* ------------------------------------------------------------------------ */
/* Interface layout for points: x[var][2][L] contiguous per point (AoS).     */
/* ------------------------------------------------------------------------ */
static cx load_cx(const double *p, int L)
{
    cx z = cx_zero();
    for (int l = 0; l < L; ++l) {
        z.re.v[l] = p[l];
        z.im.v[l] = p[L + l];
    }
    return z;
}

static void store_cx(double *p, int L, cx z)
{
    for (int l = 0; l < L; ++l) {
        p[l] = z.re.v[l];
        p[L + l] = z.im.v[l];
    }
}

typedef struct {
    int n_eq, n_var;
    const int32_t *eq_term_off, *term_fac_off, *fac_var, *fac_exp;
    const double *coef; /* [T][2], FP64 values define the system */
} sysv;

/* Total degree of each equation of f: the largest exponent sum over its terms. */
static void sys_degrees(const sysv *f, int32_t *deg)
{
    for (int i = 0; i < f->n_eq; ++i) {
        int best = 0;
        for (int s = f->eq_term_off[i]; s < f->eq_term_off[i + 1]; ++s) {
            int d = 0;
            for (int q = f->term_fac_off[s]; q < f->term_fac_off[s + 1]; ++q) d += f->fac_exp[q];
            if (d > best) best = d;
        }
        deg[i] = best;
    }
}

/* z^e by repeated multiplication, left to right. */
static cx cx_pow(int L, cx z, int e)
{
    cx r = cx_d(1.0, 0.0);
    for (int k = 0; k < e; ++k) r = cx_mul(L, r, z);
    return r;
}

/*
 * Evaluate one polynomial system (the "plain definition", Table 4 host side):
 * v_i = sum_terms c * prod_j x_j^{a_j}, and J_ij = sum_terms (a_j c) x_j^{a_j-1}
 * prod_{l != j} x_l^{a_l}, every derivative formed directly from its symbolic
 * expression.  scale multiplies every coefficient (the homotopy's c(t)).
 * Also accumulates the FP64 magnitude bounds sv_i = sum |c s| |x^a| and
 * sj_ij = sum a_j |c s| |x^(a - e_j)|.
 */
static void eval_system(int L, const sysv *f, cx scale, const cx *x, cx *val, cx *jac,
                        double *sv, double *sj)
{
    int n = f->n_var;
    double sabs = cx_absd(scale);
    for (int i = 0; i < f->n_eq; ++i) {
        for (int s = f->eq_term_off[i]; s < f->eq_term_off[i + 1]; ++s) {
            int q0 = f->term_fac_off[s], q1 = f->term_fac_off[s + 1];
            cx c = cx_mul(L, cx_d(f->coef[2 * s], f->coef[2 * s + 1]), scale);
            double cabs = hypot(f->coef[2 * s], f->coef[2 * s + 1]) * sabs;
            /* value of the term: c * x_{j1}^{a1} * x_{j2}^{a2} * ... */
            cx m = c;
            double mabs = cabs;
            for (int q = q0; q < q1; ++q) {
                for (int r = 0; r < f->fac_exp[q]; ++r) m = cx_mul(L, m, x[f->fac_var[q]]);
                mabs *= pow(cx_absd(x[f->fac_var[q]]), f->fac_exp[q]);
            }
            val[i] = cx_add(L, val[i], m);
            if (sv) sv[i] += mabs;
            if (!jac) continue;
            /* each derivative directly: (a_j c) x_j^{a_j - 1} prod_{l != j} x_l^{a_l} */
            for (int qd = q0; qd < q1; ++qd) {
                int a = f->fac_exp[qd];
                cx d = cx_scale(L, c, mp_d((double)a));
                double dabs = cabs * a;
                for (int q = q0; q < q1; ++q) {
                    int e = f->fac_exp[q] - (q == qd ? 1 : 0);
                    for (int r = 0; r < e; ++r) d = cx_mul(L, d, x[f->fac_var[q]]);
                    dabs *= pow(cx_absd(x[f->fac_var[q]]), e);
                }
                int j = f->fac_var[qd];
                jac[(size_t)i * n + j] = cx_add(L, jac[(size_t)i * n + j], d);
                if (sj) sj[(size_t)i * n + j] += dabs;
            }
        }
    }
}

/*
 * Homotopy H(x, t) = gamma (1 - t) g(x) + t f(x) of Eq. (1) and its Jacobian
 * in x.  g is either a given system or, when NULL, the total-degree start
 * system g_i = x_i^{d_i} - 1 with d_i the degree of f_i.  has_t = 0 means
 * t = 1 (f alone).  (1 - t) is formed exactly from the FP64 t.
 */
static void eval_homotopy(int L, const sysv *f, const sysv *g, const int32_t *deg, cx gamma,
                          int has_t, double t, const cx *x, cx *val, cx *jac, double *sv,
                          double *sj)
{
    int ne = f->n_eq, n = f->n_var;
    for (int i = 0; i < ne; ++i) val[i] = cx_zero();
    if (jac)
        for (int k = 0; k < ne * n; ++k) jac[k] = cx_zero();
    if (sv) memset(sv, 0, sizeof(double) * ne);
    if (sj) memset(sj, 0, sizeof(double) * ne * n);
    if (!has_t) {
        eval_system(L, f, cx_d(1.0, 0.0), x, val, jac, sv, sj);
        return;
    }
    cx tf = cx_d(t, 0.0);
    expn e;
    ex_zero(&e);
    ex_add_d(&e, 1.0);
    ex_add_d(&e, -t);
    mp omt = ex_to_mp(&e, L); /* 1 - t, exact for L >= 2 */
    cx gs = cx_scale(L, gamma, omt);
    eval_system(L, f, tf, x, val, jac, sv, sj);
    if (g) {
        eval_system(L, g, gs, x, val, jac, sv, sj);
        return;
    }
    double gabs = cx_absd(gs);
    for (int i = 0; i < ne; ++i) {
        int d = deg[i];
        cx xi = x[i];
        cx p = cx_pow(L, xi, d);
        cx gi = cx_sub(L, p, cx_d(1.0, 0.0));
        val[i] = cx_add(L, val[i], cx_mul(L, gs, gi));
        double xa = cx_absd(xi);
        if (sv) sv[i] += gabs * (pow(xa, d) + 1.0);
        if (jac) {
            cx dg = cx_scale(L, cx_pow(L, xi, d - 1), mp_d((double)d));
            jac[(size_t)i * n + i] = cx_add(L, jac[(size_t)i * n + i], cx_mul(L, gs, dg));
            if (sj) sj[(size_t)i * n + i] += gabs * d * pow(xa, d - 1);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Modified Gram-Schmidt least squares on the augmented matrix [A | b].      */
/* ------------------------------------------------------------------------ */
/*
 * A is m x n (m >= n), column-major in w[col * m + row], with b appended as
 * column n.  For k = 0..n-1: r_kk = ||w_k||, q_k = w_k / r_kk, and for every
 * later column j (including b) r_kj = q_k^H w_j, w_j -= r_kj q_k.  Then
 * R dx = (r_kn) by back substitution.  Returns 0, or 1 (singular) when some
 * r_kk <= eps_s * ||A||_F.  w is overwritten; dx has n entries.
 */
static int mgs_solve(int L, int m, int n, cx *w, cx *dx, double eps_s)
{
    cx *R = (cx *)calloc((size_t)n * (n + 1), sizeof(cx));
    double fro = 0.0;
    for (int k = 0; k < m * n; ++k) {
        double a = cx_absd(w[k]);
        fro += a * a;
    }
    fro = sqrt(fro);
    int singular = 0;
    for (int k = 0; k < n && !singular; ++k) {
        cx *wk = w + (size_t)k * m;
        mp nrm2 = mp_d(0.0);
        for (int i = 0; i < m; ++i) nrm2 = mp_add(L, nrm2, cx_abs2(L, wk[i]));
        mp rkk = mp_sqrt(L, nrm2);
        if (!(mp_hi(rkk) > eps_s * fro)) {
            singular = 1;
            break;
        }
        R[(size_t)k * (n + 1) + k].re = rkk;
        for (int i = 0; i < m; ++i) {
            wk[i].re = mp_div(L, wk[i].re, rkk);
            wk[i].im = mp_div(L, wk[i].im, rkk);
        }
        for (int j = k + 1; j <= n; ++j) {
            cx *wj = w + (size_t)j * m;
            cx r = cx_zero();
            for (int i = 0; i < m; ++i) r = cx_add(L, r, cx_cmul(L, wk[i], wj[i]));
            R[(size_t)k * (n + 1) + j] = r;
            for (int i = 0; i < m; ++i) wj[i] = cx_sub(L, wj[i], cx_mul(L, r, wk[i]));
        }
    }
    if (!singular) {
        for (int k = n - 1; k >= 0; --k) {
            cx s = R[(size_t)k * (n + 1) + n];
            for (int j = k + 1; j < n; ++j) s = cx_sub(L, s, cx_mul(L, R[(size_t)k * (n + 1) + j], dx[j]));
            mp rkk = R[(size_t)k * (n + 1) + k].re;
            dx[k].re = mp_div(L, s.re, rkk);
            dx[k].im = mp_div(L, s.im, rkk);
        }
    }
    free(R);
    return singular;
}

static double eps_singular(int L)
{
    /* 1e-13 in FP64, 2^-96 in double double, 2^-200 in quad double */
    return L == 1 ? 1e-13 : (L == 2 ? ldexp(1.0, -96) : ldexp(1.0, -200));
}

/* ------------------------------------------------------------------------ */
/* Exported API                                                              */
/* ------------------------------------------------------------------------ */

void ora_degrees(int n_eq, int n_var, const int32_t *eq_term_off, const int32_t *term_fac_off,
                 const int32_t *fac_var, const int32_t *fac_exp, const double *coef, int32_t *deg)
{
    sysv f = {n_eq, n_var, eq_term_off, term_fac_off, fac_var, fac_exp, coef};
    sys_degrees(&f, deg);
}

/* Arithmetic probes for the pins: op 0 add, 1 sub, 2 mul, 3 div, 4 sqrt(a). */
void ora_mp_op(int L, int op, const double *a, const double *b, double *out)
{
    mp x = mp_d(0.0), y = mp_d(0.0), r;
    for (int l = 0; l < L; ++l) {
        x.v[l] = a[l];
        y.v[l] = b ? b[l] : 0.0;
    }
    switch (op) {
    case 0: r = mp_add(L, x, y); break;
    case 1: r = mp_sub(L, x, y); break;
    case 2: r = mp_mul(L, x, y); break;
    case 3: r = mp_div(L, x, y); break;
    default: r = mp_sqrt(L, x); break;
    }
    for (int l = 0; l < L; ++l) out[l] = r.v[l];
}

/* Complex probes: op 0 add, 1 mul, 2 conj(a)*b. a, b, out are [2][L]. */
void ora_cx_op(int L, int op, const double *a, const double *b, double *out)
{
    cx x = load_cx(a, L), y = load_cx(b, L), r;
    switch (op) {
    case 0: r = cx_add(L, x, y); break;
    case 1: r = cx_mul(L, x, y); break;
    default: r = cx_cmul(L, x, y); break;
    }
    store_cx(out, L, r);
}

/*
 * Evaluate H and its Jacobian at npts points.  x is [npts][n_var][2][L],
 * val [npts][n_eq][2][L], jac [npts][n_eq][n_var][2][L] (nullable),
 * sv [npts][n_eq], sj [npts][n_eq][n_var] (nullable).  g == NULL selects the
 * total-degree start system; has_t == 0 evaluates f alone.
 */
void ora_eval(int L, int n_eq, int n_var, const int32_t *eq_term_off,
              const int32_t *term_fac_off, const int32_t *fac_var, const int32_t *fac_exp,
              const double *coef, int g_present, const int32_t *g_eq_term_off,
              const int32_t *g_term_fac_off, const int32_t *g_fac_var, const int32_t *g_fac_exp,
              const double *g_coef, const double *gamma, int has_t, const double *t, int64_t npts,
              const double *x, double *val, double *jac, double *sv, double *sj)
{
    sysv f = {n_eq, n_var, eq_term_off, term_fac_off, fac_var, fac_exp, coef};
    sysv g = {n_eq, n_var, g_eq_term_off, g_term_fac_off, g_fac_var, g_fac_exp, g_coef};
    int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * n_eq);
    sys_degrees(&f, deg);
    cx *xp = (cx *)malloc(sizeof(cx) * n_var);
    cx *vp = (cx *)malloc(sizeof(cx) * n_eq);
    cx *jp = jac ? (cx *)malloc(sizeof(cx) * n_eq * n_var) : NULL;
    cx gam = cx_d(gamma[0], gamma[1]);
    size_t xs = (size_t)n_var * 2 * L, vs = (size_t)n_eq * 2 * L;
    for (int64_t p = 0; p < npts; ++p) {
        for (int j = 0; j < n_var; ++j) xp[j] = load_cx(x + p * xs + (size_t)j * 2 * L, L);
        eval_homotopy(L, &f, g_present ? &g : NULL, deg, gam, has_t, has_t ? t[p] : 1.0, xp, vp,
                      jp, sv ? sv + p * n_eq : NULL, sj ? sj + p * (size_t)n_eq * n_var : NULL);
        for (int i = 0; i < n_eq; ++i) store_cx(val + p * vs + (size_t)i * 2 * L, L, vp[i]);
        if (jac)
            for (int k = 0; k < n_eq * n_var; ++k)
                store_cx(jac + p * vs * n_var + (size_t)k * 2 * L, L, jp[k]);
    }
    free(deg);
    free(xp);
    free(vp);
    free(jp);
}

/*
 * Least squares by MGS on one m x n complex system A dx = b, L limbs.
 * A is [m][n][2][L] row-major, b [m][2][L], dx [n][2][L].  Returns 1 if
 * singular.  q_out (nullable, [m][n][2][L]) receives the orthonormal Q.
 */
int ora_mgs(int L, int m, int n, const double *A, const double *b, double *dx, double *q_out)
{
    cx *w = (cx *)malloc(sizeof(cx) * (size_t)m * (n + 1));
    cx *d = (cx *)malloc(sizeof(cx) * n);
    for (int i = 0; i < m; ++i) {
        for (int j = 0; j < n; ++j) w[(size_t)j * m + i] = load_cx(A + ((size_t)i * n + j) * 2 * L, L);
        w[(size_t)n * m + i] = load_cx(b + (size_t)i * 2 * L, L);
    }
    int sing = mgs_solve(L, m, n, w, d, eps_singular(L));
    if (!sing) {
        for (int j = 0; j < n; ++j) store_cx(dx + (size_t)j * 2 * L, L, d[j]);
        if (q_out)
            for (int i = 0; i < m; ++i)
                for (int j = 0; j < n; ++j) store_cx(q_out + ((size_t)i * n + j) * 2 * L, L, w[(size_t)j * m + i]);
    }
    free(w);
    free(d);
    return sing;
}

/* ------------------------------------------------------------------------ */
/* Start solutions of g_i = x_i^{d_i} - 1                                    */
/* ------------------------------------------------------------------------ */
/*
 * Path p maps to the multi-index (k_0, ..., k_{n-1}) by little-endian mixed
 * radix, p = sum k_i prod_{l<i} d_l, and x_i = exp(2 pi i k_i / d_i).  Only
 * d in {1, 2, 3, 4, 6} has a closed form here (enough for every workload):
 * cos/sin of multiples of pi/2 and pi/3, with sqrt(3)/2 formed in L limbs.
 */
static int root_of_unity(int L, int d, int k, cx *out)
{
    if (d <= 0 || 12 % d != 0 || d == 12) return 1;
    k %= d;
    int a = ((12 / d) * k) % 12; /* angle 2 pi k / d in units of 30 degrees */
    mp h3 = mp_sqrt(L, mp_d(3.0));
    for (int l = 0; l < L; ++l) h3.v[l] *= 0.5; /* sqrt(3)/2, exact halving */
    mp zero = mp_d(0.0), one = mp_d(1.0), half = mp_d(0.5);
    mp c, s;
    switch (a) {
    case 0: c = one; s = zero; break;
    case 2: c = half; s = h3; break;
    case 3: c = zero; s = one; break;
    case 4: c = mp_neg(L, half); s = h3; break;
    case 6: c = mp_neg(L, one); s = zero; break;
    case 8: c = mp_neg(L, half); s = mp_neg(L, h3); break;
    case 9: c = zero; s = mp_neg(L, one); break;
    case 10: c = half; s = mp_neg(L, h3); break;
    default: return 1;
    }
    out->re = c;
    out->im = s;
    return 0;
}

int ora_start_solution(int L, int n, const int32_t *deg, int64_t p, double *x /* [n][2][L] */)
{
    for (int i = 0; i < n; ++i) {
        int k = (int)(p % deg[i]);
        p /= deg[i];
        cx z;
        if (root_of_unity(L, deg[i], k, &z)) return 1;
        store_cx(x + (size_t)i * 2 * L, L, z);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Path tracker (Section 2, Tables 1-3)                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t prec, mixed, predictor_order, max_newton, expand_after, polish_max;
    double h_init, h_min, h_max, shrink, expand, tol_dx, diverge_norm, polish_tol;
    int64_t max_steps;
    double tol_res;
} ora_opts;

enum { R_NONE = 0, R_SUCCESS = 1, R_DIVERGED = 2, R_STEP_UNDERFLOW = 3, R_MAX_STEPS = 4,
       R_SINGULAR = 5, R_NAN = 6 };

static double norm_inf(int n, const cx *x)
{
    double m = 0.0;
    for (int j = 0; j < n; ++j) {
        double a = cx_absd(x[j]);
        if (isnan(a)) return a;
        if (a > m) m = a;
    }
    return m;
}

static int has_nan(int n, const cx *x)
{
    for (int j = 0; j < n; ++j)
        if (isnan(x[j].re.v[0]) || isnan(x[j].im.v[0]) || isinf(x[j].re.v[0]) || isinf(x[j].im.v[0]))
            return 1;
    return 0;
}

/* One Newton step at (x, t): solve J dx = -H by MGS (FP64 when mixed, else
 * L limbs) and return dx.  Returns 1 when MGS flags the matrix singular.
 * hres (nullable) receives ||H(x, t)||_inf and jfro (nullable) ||J||_F, both
 * from the leading limbs in FP64: the residual at the point where the Newton
 * system is formed, and the scale it is compared against. */
static int newton_step(int L, int mixed, const sysv *f, const sysv *g, const int32_t *deg, cx gamma,
                       int has_t, double t, const cx *x, cx *dx, cx *hv, cx *jm, cx *w,
                       double *hres, double *jfro)
{
    int n = f->n_var, m = f->n_eq;
    eval_homotopy(L, f, g, deg, gamma, has_t, t, x, hv, jm, NULL, NULL);
    if (hres) *hres = norm_inf(m, hv);
    if (jfro) {
        double s = 0.0;
        for (int k = 0; k < m * n; ++k) s += jm[k].re.v[0] * jm[k].re.v[0] + jm[k].im.v[0] * jm[k].im.v[0];
        *jfro = sqrt(s);
    }
    int Ls = mixed ? 1 : L;
    for (int i = 0; i < m; ++i) {
        for (int j = 0; j < n; ++j) {
            cx a = jm[(size_t)i * n + j];
            if (mixed) a = cx_d(a.re.v[0], a.im.v[0]);
            w[(size_t)j * m + i] = a;
        }
        cx r = hv[i];
        r.re = mp_neg(L, r.re);
        r.im = mp_neg(L, r.im);
        if (mixed) r = cx_d(r.re.v[0], r.im.v[0]);
        w[(size_t)n * m + i] = r;
    }
    int sing = mgs_solve(Ls, m, n, w, dx, eps_singular(Ls));
    if (mixed && !sing)
        for (int j = 0; j < n; ++j) dx[j] = cx_d(dx[j].re.v[0], dx[j].im.v[0]);
    return sing;
}

/*
 * Predictor of order m >= 2 (Section 2: an extrapolation applied to each
 * coordinate separately; a fourth-order predictor uses the current and four
 * previous points): the value at t1 of the polynomial of degree m in t that
 * interpolates (T[j], X[j]), j = 0..m, written in Lagrange form.  The weights
 * are formed in FP64, w_j = prod_{i != j} (t1 - T_i) / (T_j - T_i) with the
 * factors taken in increasing i, and the sum over j in increasing j is
 * formed in L limbs.  X is [m+1][n] (X[0] the current point).
 */
static void lagrange_weights(int m, const double *T, double t1, double *w)
{
    for (int j = 0; j <= m; ++j) {
        double wj = 1.0;
        for (int i = 0; i <= m; ++i) {
            if (i == j) continue;
            double num = t1 - T[i];
            double den = T[j] - T[i];
            wj = wj * (num / den);
        }
        w[j] = wj;
    }
}

static void extrapolate(int L, int m, int n, const double *T, cx *const *X, double t1, cx *out)
{
    double w[8];
    lagrange_weights(m, T, t1, w);
    for (int k = 0; k < n; ++k) {
        cx acc = cx_scale(L, X[0][k], mp_d(w[0]));
        for (int j = 1; j <= m; ++j) acc = cx_add(L, acc, cx_scale(L, X[j][k], mp_d(w[j])));
        out[k] = acc;
    }
}

/* Exported for the pins: out = p(t1) for the interpolant of (T[j], X[j]),
 * X as [m+1][n][2][L]. */
void ora_extrapolate(int L, int m, int n, const double *T, const double *X, double t1, double *out)
{
    cx *buf = (cx *)malloc(sizeof(cx) * (size_t)(m + 1) * n);
    cx *rows[8];
    for (int j = 0; j <= m; ++j) {
        rows[j] = buf + (size_t)j * n;
        for (int k = 0; k < n; ++k) rows[j][k] = load_cx(X + ((size_t)j * n + k) * 2 * L, L);
    }
    cx *o = (cx *)malloc(sizeof(cx) * n);
    extrapolate(L, m, n, T, rows, t1, o);
    for (int k = 0; k < n; ++k) store_cx(out + (size_t)k * 2 * L, L, o[k]);
    free(o);
    free(buf);
}

/*
 * Track one path from x (a start solution of g, t = 0) to t = 1 (Section 2).
 * Step control: h <- min(h, 1 - t); predict (with predictor_order 1 the
 * secant through the last two accepted points; with order m >= 2 the
 * extrapolation above through the current point and up to m previous
 * accepted points, the secant while only one previous point exists; the
 * current point on the first step); then evaluate-correct with at most
 * max_newton Newton steps.  Section 2 ends the corrector when both the
 * residuals and the size of the updates are small: a step converges when
 * ||dx|| <= tol_dx max(1, ||x||) and the residual at the point where the
 * Newton system was formed satisfies ||H|| <= tol_res ||J||_F max(1, ||x||)
 * (x the updated point, every norm in FP64 from the leading limbs); it fails
 * when a later update does not shrink or MGS is singular.  Accepted steps
 * advance t and count toward expansion of h (x expand after expand_after
 * successes, capped by h_max); rejected ones shrink h and fail below h_min.
 * At t = 1 the endpoint is polished by Newton on f in the residual precision
 * (a non-finite update is never applied); a polished endpoint that is not
 * finite, or lies beyond diverge_norm, ends the path as a failure.
 * g_present = 0 selects the total-degree start system g_i = x_i^{d_i} - 1.
 */
int ora_track_path(int L, const ora_opts *o, int n_eq, int n_var, const int32_t *eq_term_off,
                   const int32_t *term_fac_off, const int32_t *fac_var, const int32_t *fac_exp,
                   const double *coef, int g_present, const int32_t *g_eq_term_off,
                   const int32_t *g_term_fac_off, const int32_t *g_fac_var,
                   const int32_t *g_fac_exp, const double *g_coef, const double *gamma,
                   double *x_io /* [n][2][L] */, int32_t *reason_out, int64_t *steps_out,
                   int64_t *rejected_out, int64_t *newton_out, double *t_out)
{
    sysv f = {n_eq, n_var, eq_term_off, term_fac_off, fac_var, fac_exp, coef};
    sysv gs = {n_eq, n_var, g_eq_term_off, g_term_fac_off, g_fac_var, g_fac_exp, g_coef};
    const sysv *g = g_present ? &gs : NULL;
    int n = n_var, m = n_eq;
    int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * m);
    sys_degrees(&f, deg);
    cx gam = cx_d(gamma[0], gamma[1]);
    cx *x = (cx *)malloc(sizeof(cx) * n), *xp = (cx *)malloc(sizeof(cx) * n);
    /* older accepted points for predictor orders 2..4: xq[0] is the one
     * before xp, xq[2] the oldest */
    cx *xq[3];
    double tq[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < 3; ++q) xq[q] = (cx *)malloc(sizeof(cx) * n);
    const int order = o->predictor_order < 1 ? 1 : (o->predictor_order > 4 ? 4 : o->predictor_order);
    int nh = 0; /* accepted points before the current one that are kept */
    cx *xh = (cx *)malloc(sizeof(cx) * n), *dx = (cx *)malloc(sizeof(cx) * n);
    cx *hv = (cx *)malloc(sizeof(cx) * m), *jm = (cx *)malloc(sizeof(cx) * m * n);
    cx *w = (cx *)malloc(sizeof(cx) * m * (n + 1));
    for (int j = 0; j < n; ++j) x[j] = load_cx(x_io + (size_t)j * 2 * L, L);
    double t = 0.0, tp = 0.0, h = o->h_init;
    int have_prev = 0, succ = 0, reason = R_NONE;
    int64_t steps = 0, rejected = 0, newton = 0;
    if (has_nan(n, x)) reason = R_NAN;
    if (o->h_min > o->h_init) reason = R_STEP_UNDERFLOW;
    while (reason == R_NONE) {
        if (steps >= o->max_steps) {
            reason = R_MAX_STEPS;
            break;
        }
        steps++;
        if (h > 1.0 - t) h = 1.0 - t;
        double t1 = t + h;
        if (t1 >= 1.0 - 1e-15) t1 = 1.0;
        /* predict */
        const int mo = nh < order ? nh : order;
        if (mo >= 2) {
            double T[5] = {t, tp, tq[0], tq[1], tq[2]};
            cx *X[5] = {x, xp, xq[0], xq[1], xq[2]};
            extrapolate(L, mo, n, T, X, t1, xh);
        } else if (have_prev) {
            double r = (t1 - t) / (t - tp);
            mp rr = mp_d(r);
            for (int j = 0; j < n; ++j) xh[j] = cx_add(L, x[j], cx_scale(L, cx_sub(L, x[j], xp[j]), rr));
        } else {
            for (int j = 0; j < n; ++j) xh[j] = x[j];
        }
        /* correct */
        int conv = 0, sing = 0;
        double dprev = 0.0;
        for (int it = 1; it <= o->max_newton; ++it) {
            newton++;
            double hres = 0.0, jfro = 0.0;
            sing = newton_step(L, o->mixed, &f, g, deg, gam, 1, t1, xh, dx, hv, jm, w, &hres, &jfro);
            if (sing) break;
            for (int j = 0; j < n; ++j) xh[j] = cx_add(L, xh[j], dx[j]);
            double dn = norm_inf(n, dx), xn = norm_inf(n, xh);
            if (isnan(dn) || isnan(xn)) break;
            const double sx = xn > 1.0 ? xn : 1.0;
            if (dn <= o->tol_dx * sx && hres <= o->tol_res * jfro * sx) {
                conv = 1;
                break;
            }
            if (it >= 2 && dn > dprev) break;
            dprev = dn;
        }
        if (conv) {
            if (order >= 2) {
                cx *oldest = xq[2];
                xq[2] = xq[1];
                xq[1] = xq[0];
                xq[0] = oldest;
                for (int j = 0; j < n; ++j) xq[0][j] = xp[j];
                tq[2] = tq[1];
                tq[1] = tq[0];
                tq[0] = tp;
            }
            tp = t;
            for (int j = 0; j < n; ++j) xp[j] = x[j];
            have_prev = 1;
            if (nh < 4) nh++;
            t = t1;
            for (int j = 0; j < n; ++j) x[j] = xh[j];
            if (++succ >= o->expand_after) {
                h = h * o->expand;
                if (h > o->h_max) h = o->h_max;
                succ = 0;
            }
            if (t == 1.0) reason = R_SUCCESS;
        } else {
            rejected++;
            h *= o->shrink;
            succ = 0;
            /* a step size below h_min ends the path; when the last rejection
             * came from a rank-deficient Jacobian the cause is reported */
            if (h < o->h_min) reason = sing ? R_SINGULAR : R_STEP_UNDERFLOW;
        }
        if (reason == R_NONE || reason == R_SUCCESS) {
            if (has_nan(n, x)) reason = R_NAN;
            else if (norm_inf(n, x) > o->diverge_norm) reason = R_DIVERGED;
        }
    }
    if (reason == R_SUCCESS) {
        /* polish at t = 1: Newton on f until ||dx|| <= polish_tol max(1,||x||)
         * or the update stops halving, at most polish_max steps; an update
         * that is not finite ends the polish without being applied */
        double dprev = INFINITY;
        for (int it = 0; it < o->polish_max; ++it) {
            int sing = newton_step(L, o->mixed, &f, g, deg, gam, 0, 1.0, x, dx, hv, jm, w, NULL, NULL);
            if (sing) break;
            double dn = norm_inf(n, dx);
            if (!isfinite(dn)) break;
            if (!(dn < 0.5 * dprev) && it > 0) break;
            for (int j = 0; j < n; ++j) x[j] = cx_add(L, x[j], dx[j]);
            newton++;
            double xn = norm_inf(n, x);
            if (dn <= o->polish_tol * (xn > 1.0 ? xn : 1.0)) break;
            dprev = dn;
        }
        /* the endpoint must be finite and within diverge_norm */
        if (has_nan(n, x)) reason = R_NAN;
        else if (norm_inf(n, x) > o->diverge_norm) reason = R_DIVERGED;
    }
    for (int j = 0; j < n; ++j) store_cx(x_io + (size_t)j * 2 * L, L, x[j]);
    if (reason_out) *reason_out = reason;
    if (steps_out) *steps_out = steps;
    if (rejected_out) *rejected_out = rejected;
    if (newton_out) *newton_out = newton;
    if (t_out) *t_out = t;
    free(deg); free(x); free(xp); free(xh); free(dx); free(hv); free(jm); free(w);
    for (int q = 0; q < 3; ++q) free(xq[q]);
    return reason == R_SUCCESS ? 1 : -1;
}
