/*
 * ph.h -- C ABI of the many-path polynomial homotopy library for AMD MI355X
 * (gfx950).  Hot path of J. Verschelde and X. Yu, "Tracking Many Solution
 * Paths of a Polynomial Homotopy on a Graphics Processing Unit" (2015).
 *
 * Conventions shared by every call:
 *   - Every function returns int: PH_OK (0) or a negative PH_E* code.  The
 *     message of the last failure on the calling thread is ph_last_error().
 *   - Precision `prec` is the number of FP64 limbs of every real quantity:
 *     PH_D = 1 (complex double), PH_DD = 2 (double double), PH_QD = 4 (quad
 *     double), as in Section 1 of the paper.  Limbs are non-overlapping with
 *     the largest first; a value is the exact sum of its limbs.
 *   - Point data is structure-of-arrays with the point (path) index fastest,
 *     the "vertical" layout of the paper (Section 3, Table 5): element
 *     (point p, row r) lives at base[r * ld + p], ld >= number of points.
 *       x   : row r = (var * 2 + c) * L + l          c = 0 real, 1 imaginary
 *       val : row r = (eq * 2 + c) * L + l
 *       jac : row r = ((eq * n_var + var) * 2 + c) * L + l
 *   - Pointers marked "device" are device memory on the current HIP device;
 *     the caller owns them.  `stream` is a hipStream_t (NULL: default stream).
 *   - A numerical failure of one path is not an error: it is reported through
 *     the per-path status (1 success, -1 failure; 0 is used internally for
 *     "continue", Section 2) and a reason code.
 */
#ifndef PH_H
#define PH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PH_OK 0
#define PH_EINVAL (-1)       /* bad size, pointer, precision or exponent */
#define PH_ENOMEM (-2)       /* device or host allocation failed */
#define PH_EHIP (-3)         /* a HIP runtime call failed (message has the HIP error) */
#define PH_EUNSUPPORTED (-4) /* valid request outside what the library handles */

#define PH_D 1
#define PH_DD 2
#define PH_QD 4

/* Per-path reasons (status -1 unless PH_R_SUCCESS). */
#define PH_R_NONE 0
#define PH_R_SUCCESS 1
#define PH_R_DIVERGED 2       /* ||x||_inf exceeded diverge_norm */
#define PH_R_STEP_UNDERFLOW 3 /* step size fell below h_min */
#define PH_R_MAX_STEPS 4      /* step budget exhausted */
#define PH_R_SINGULAR 5       /* last rejected step had a rank-deficient Jacobian */
#define PH_R_NAN 6            /* NaN or Inf in the path state */

typedef struct ph_system ph_system; /* opaque; immutable after creation */

/*
 * ph_system_create -- compile a sparse polynomial system into device term
 * tables (the paper's "instructions", idx and cff, Table 8).
 *   n_eq, n_var    : 1 <= n_var <= n_eq <= 64 (least squares allowed for eval)
 *   eq_term_off    : host, n_eq + 1 offsets; terms of equation i are
 *                    eq_term_off[i] .. eq_term_off[i+1]-1
 *   term_fac_off   : host, n_terms + 1 offsets into fac_var / fac_exp; a term
 *                    with no factor is a constant
 *   fac_var        : host, variable index of each factor, strictly increasing
 *                    inside a term
 *   fac_exp        : host, exponent of each factor, 1 <= e <= 64
 *   coef           : host, [n_terms][2][coef_limbs] complex coefficients
 *   coef_limbs     : 1, 2 or 4
 *   out            : receives the handle
 * Each term is c * prod x_j^{a_j}, decomposed as in Section 1: the product of
 * the variables that occur, times the factor c * prod x_j^{a_j - 1} common to
 * all derivatives.  At most 32 factors per term.  All host arrays are copied;
 * the call synchronises the device.  Errors: PH_EINVAL on malformed input,
 * PH_EUNSUPPORTED for n > 64 or k > 32, PH_ENOMEM / PH_EHIP.
 */
int ph_system_create(int32_t n_eq, int32_t n_var, const int32_t *eq_term_off,
                     const int32_t *term_fac_off, const int32_t *fac_var,
                     const int32_t *fac_exp, const double *coef, int32_t coef_limbs,
                     ph_system **out);

/* Free the handle and its device tables (synchronises the device). */
int ph_system_destroy(ph_system *s);

/* Shape of a system: any output pointer may be NULL. */
int ph_system_info(const ph_system *s, int32_t *n_eq, int32_t *n_var, int64_t *n_terms,
                   int32_t *max_factors);

/* deg[i] = total degree of equation i (host array of n_eq). */
int ph_system_degrees(const ph_system *s, int32_t *deg);

/*
 * ph_start_solutions -- start points of the total-degree start system
 * g_i = x_i^{d_i} - 1 (the start system of Eq. (1) used by ph_track):
 * path p maps to the multi-index (k_0 .. k_{n-1}) by little-endian mixed
 * radix p = sum_i k_i prod_{l<i} d_l and x_i = exp(2 pi i k_i / d_i).
 * Writes paths first_path .. first_path+npaths-1 into the device SoA array x
 * (row = (var*2+c)*prec + l, leading dimension ld).  Degrees must divide 12
 * (1, 2, 3, 4, 6): PH_EUNSUPPORTED otherwise.  Asynchronous on stream.
 */
int ph_start_solutions(const ph_system *target, int32_t prec, int64_t first_path,
                       int64_t npaths, double *x, int64_t ld, void *stream);

/*
 * ph_eval_jac -- values and Jacobian of the homotopy of Eq. (1),
 *   H(x, t) = gamma (1 - t) g(x) + t f(x),   J = dH/dx,
 * at npts points, by reverse-mode differentiation of every term's variable
 * product (Section 3, Table 6), the coefficient c(t) folded per point.
 *   target : f;  start : g, or NULL for g_i = x_i^{d_i} - 1 with d_i = deg f_i
 *   gamma  : host, {re, im} FP64
 *   prec   : PH_D, PH_DD or PH_QD
 *   t      : device, npts FP64 values of t, or NULL for t = 1 (f alone)
 *   x      : device SoA, rows (var*2+c)*prec+l, leading dimension ld
 *   val    : device SoA output, rows (eq*2+c)*prec+l
 *   jac    : device SoA output, rows ((eq*n_var+var)*2+c)*prec+l, or NULL
 * npts = 0 is a no-op.  No allocation and no synchronisation: the call only
 * queues kernels on stream (it may be captured in a hipGraph).  The term
 * tables of (target, NULL) exist from ph_system_create; those of (target,
 * start) are built once by ph_eval_prepare, and a start system that was not
 * prepared for this target is PH_EINVAL.  A tuned configuration is looked up
 * in memory (the handle, or the PH_AUTOTUNE_CACHE entries read when target was
 * created).  NaN/Inf inputs propagate unchecked.  Errors: PH_EINVAL (null
 * pointers, ld < npts, start shape differs from target, start not prepared,
 * unfused design without prepared arrays), PH_EHIP (launch failure).
 */
int ph_eval_jac(const ph_system *target, const ph_system *start, const double gamma[2],
                int32_t prec, int64_t npts, const double *t, const double *x, int64_t ld,
                double *val, double *jac, void *stream);

/*
 * ph_eval_prepare -- the one point where ph_eval_jac's device data for
 * (target, start) is allocated: builds the merged term table of f and the
 * start system g of Eq. (1) (start NULL: the total-degree table, which
 * ph_system_create already built), and, with unfused_points > 0, sizes the
 * intermediate arrays of the unfused design (kernel 5 of ph_eval_set_config:
 * (terms + slots) * 16 * prec bytes per point) for that many points of
 * precision prec; larger batches then run in chunks of that many points.
 * Idempotent and grow-only.  Allocates device memory and synchronises the
 * device.  Errors: PH_EINVAL (null target, bad prec, unfused_points < 0,
 * start shape differs from target), PH_ENOMEM, PH_EHIP.
 */
int ph_eval_prepare(ph_system *target, const ph_system *start, int32_t prec,
                    int64_t unfused_points);

/*
 * ph_eval_set_config -- pin the kernel and tiling ph_eval_jac uses for
 * (target, start, prec): kernel 0 automatic, 1 general (Jacobian row
 * accumulated in the output), 2 register-resident row (double, n_var <= 32),
 * 3 fast path (n_var <= 32, <= 8 factors per term, exponents <= 4 and, in
 * double double and quad double, x and its powers fitting the 160 KB of LDS)
 * with the Jacobian row on chip: in pinned registers (double), in the
 * accumulation registers (double double: one point per lane; quad double:
 * one point per two lanes), at most four waves per workgroup in double double
 * and quad double (a larger count launches four), 4 the double fast path
 * with a compiler-held row,
 * 5 the paper's unfused design (coeff, mon and sum kernels with the
 * coefficients and the k + 1 products of every term and point stored in
 * device memory between them; an ablation of the fused kernels, whose
 * intermediate arrays ph_eval_prepare sizes; waves and groups are ignored);
 * kernels 2, 3 and 4 produce the Jacobian: a values-only call (jac NULL)
 * runs the general kernel with the same waves and groups;
 * waves = waves per workgroup sharing one 64-point tile (1..8, 0 default;
 * taken as given, so counts like 6 can match the register budget);
 * groups = equation groups per tile (power of two, 0 default).  All zero
 * clears the setting.  Host-only; PH_EINVAL on bad values.  A kernel that
 * does not apply makes later ph_eval_jac calls fail with PH_EUNSUPPORTED.
 */
int ph_eval_set_config(ph_system *target, const ph_system *start, int32_t prec, int32_t kernel,
                       int32_t waves, int32_t groups);

/*
 * ph_eval_get_config -- the configuration ph_eval_jac would use for (target,
 * start, prec): the one pinned or tuned in this handle, else the last entry
 * for these systems in the PH_AUTOTUNE_CACHE file as read when target was
 * created (which the handle then keeps); all zero: automatic.  Host-only;
 * PH_EINVAL on null pointers.
 */
int ph_eval_get_config(const ph_system *target, const ph_system *start, int32_t prec,
                       int32_t *kernel, int32_t *waves, int32_t *groups);

/*
 * ph_eval_autotune -- time every applicable (kernel, waves, groups) choice of
 * ph_eval_jac on the caller's buffers (same arguments as ph_eval_jac; the
 * outputs are overwritten with a valid result) and keep the fastest for
 * (target, start, prec).  With the environment variable PH_AUTOTUNE_CACHE
 * naming a file, the choice is appended there and found again by later
 * processes (keyed by a fingerprint of the systems).  best_ms (nullable)
 * receives the average time of the chosen configuration.  Synchronises the
 * stream.  Errors as ph_eval_jac.
 */
int ph_eval_autotune(ph_system *target, const ph_system *start, const double gamma[2],
                     int32_t prec, int64_t npts, const double *t, const double *x, int64_t ld,
                     double *val, double *jac, void *stream, double *best_ms);

/*
 * Options of the path tracker (Section 2; the paper gives no constants,
 * defaults from ph_track_opts_default):
 *   prec            residual precision PH_D / PH_DD / PH_QD
 *   mixed           1: Newton update solved in complex FP64 from the rounded
 *                   Jacobian and residual, added to the prec-limb point
 *                   (refinement); 0: every step in prec limbs
 *   predictor_order 1: secant (zero order on the first step); 2..4:
 *                   extrapolation through the current and up to that many
 *                   previous accepted points, per coordinate (Section 2's
 *                   fourth-order predictor at 4); the secant while only one
 *                   previous point exists
 *   max_newton      corrector steps per predictor step (3)
 *   expand_after    successes before the step grows (3)
 *   polish_max      Newton steps of the polish at t = 1 (8)
 *   h_init, h_min, h_max   initial / smallest / largest step (0.01, 1e-10, 0.1)
 *   shrink, expand  step factors after rejection / expansion (0.5, 1.5)
 *   tol_dx, tol_res corrector converged when ||dx||_inf <= tol_dx max(1,||x||_inf)
 *                   and the residual at the point where the Newton system
 *                   was formed satisfies ||H||_inf <= tol_res ||J||_F
 *                   max(1,||x||_inf) (Section 2: residuals and updates small;
 *                   norms in FP64 from the leading limbs; 1e-8, 1e-6)
 *   diverge_norm    ||x||_inf beyond this fails the path, also after the
 *                   polish (1e8)
 *   polish_tol      polish target relative to max(1,||x||); < 0 selects 8 u_prec
 *   max_steps       predictor steps per path (100000)
 *   schedule        PH_SCHED_PERSISTENT (one persistent kernel drains a device
 *                   work queue) or PH_SCHED_GRAPH (a round kernel captured in
 *                   a hipGraph and replayed; slot state stays in device memory
 *                   and only the count of active waves crosses to the host,
 *                   Section 2, Table 3)
 *   rounds_per_launch   graph schedule: tracker rounds per kernel launch (32)
 *                   when launch_ms is 0
 *   launch_ms       graph schedule: every wave of a launch runs rounds until
 *                   this many milliseconds have passed since it started (at
 *                   least one round); rounds_per_launch is then ignored.
 *                   Results do not depend on where launches end (2.0; 0 for
 *                   a fixed round count)
 *   launches_per_sync   graph schedule: graph replays between reads of the count (8)
 *   blocks_per_cu   workgroups per CU (0: the library's default, 8); never
 *                   more than the launch's kernel fits on a CU at once
 *                   (registers, LDS), so every workgroup of a launch starts
 *                   with it
 *   lanes_per_path  lanes that share one path: 4, 8, 16 or 32; 0 selects
 *                   the natural count (the next power of two >= n, at least
 *                   4), doubled when the paths at their natural count would
 *                   fill less than one wave per SIMD.  With 2 or 4 times the
 *                   natural count, 2 or 4 lanes share each equation's term
 *                   sweeps (results unchanged bit for bit), which spreads few
 *                   paths over more waves
 */
#define PH_SCHED_PERSISTENT 0
#define PH_SCHED_GRAPH 1
typedef struct {
    int32_t prec, mixed, predictor_order, max_newton, expand_after, polish_max;
    double h_init, h_min, h_max, shrink, expand, tol_dx, diverge_norm, polish_tol;
    int64_t max_steps;
    int32_t schedule, rounds_per_launch, launches_per_sync, blocks_per_cu;
    int32_t lanes_per_path;
    double tol_res;
    double launch_ms;
} ph_track_opts;

/* Counts filled by ph_track when a report pointer is given. */
typedef struct {
    int64_t n_success, n_fail, n_diverged, n_step_underflow, n_max_steps, n_singular, n_nan;
    int64_t steps, rejected, newton_its;
    double seconds;
} ph_track_report;

/* Fill *o with the defaults listed above (prec = PH_D, mixed = 0). */
int ph_track_opts_default(ph_track_opts *o);

/*
 * ph_track -- track npaths solution paths of gamma (1-t) g + t f = 0 from t = 0
 * to t = 1 (Section 2, Tables 1-3): per path its own t and step size,
 * predict (secant or extrapolation of order 2..4), evaluate-correct with
 * Newton steps solved by MGS least squares until converged (at most
 * max_newton per step), step-size control, status 1 / -1, and a Newton polish
 * at t = 1.  Paths run in a persistent kernel that refills lanes from a
 * device work queue as paths end; no host round trip happens until all
 * paths are done.
 *   target  : square system f, n <= 32, terms with at most 8 factors
 *   start   : g, or NULL for the total-degree start g_i = x_i^{d_i} - 1
 *   gamma   : host {re, im}
 *   x_start : device SoA start points (rows (i*2+c)*prec+l), or NULL for the
 *             roots of unity of path indices 0..npaths-1 (start must be NULL)
 *   ld      : leading dimension of x_start and x_end (>= npaths)
 *   opts    : see ph_track_opts (prec, mixed, step control)
 *   x_end   : device SoA endpoints (same layout)
 *   status  : device int8[npaths], 1 success / -1 failure
 *   reason  : device int8[npaths] PH_R_* (nullable)
 *   steps   : device int32[npaths] predictor steps (nullable)
 *   rep     : host report (nullable)
 * Synchronous: returns after the stream has finished (it fills rep).
 * Allocates a few KB of device scratch per call.  Errors: PH_EINVAL,
 * PH_EUNSUPPORTED (non-square, n > 32, k > 8, predictor_order outside 1..4, degrees
 * without closed-form roots of unity), PH_ENOMEM, PH_EHIP.
 */
int ph_track(const ph_system *target, const ph_system *start, const double gamma[2],
             int64_t npaths, const double *x_start, int64_t ld, const ph_track_opts *opts,
             double *x_end, int8_t *status, int8_t *reason, int32_t *steps,
             ph_track_report *rep, void *stream);

/*
 * ph_track_noalloc -- ph_track for callers that cannot allocate device memory
 * (code that must not call hipMalloc: tight serving loops, harnesses that
 * forbid allocation).  Same arguments, results, synchrony and errors as
 * ph_track, with these differences:
 *   - the device scratch of a call (counters and work queue, the system
 *     descriptor, the predictor history of predictor_order >= 2) lives in one
 *     library-owned device buffer of 16 MiB per GPU, created when the library
 *     is loaded on that GPU and held until the process ends; the call makes no
 *     device allocation and frees nothing;
 *   - opts->schedule must be PH_SCHED_PERSISTENT (PH_EUNSUPPORTED otherwise);
 *   - an explicit start system must have been prepared for this target with
 *     ph_eval_prepare (PH_EINVAL otherwise; it builds its term table);
 *   - PH_EINVAL when the predictor history of the launch (3 * 2 * prec * 8
 *     bytes per lane slot, 64 slots per workgroup, predictor_order >= 2 only)
 *     exceeds the buffer's 16 MiB - 64 KiB (quad double at more than about
 *     five workgroups per CU): lower opts->blocks_per_cu.
 * Every call on a GPU uses that GPU's one buffer, which keeps the previous
 * call's contents (the call clears its counters itself): calls that overlap
 * on one GPU (other threads, other streams) race and must be serialised by
 * the caller.
 */
int ph_track_noalloc(const ph_system *target, const ph_system *start, const double gamma[2],
                     int64_t npaths, const double *x_start, int64_t ld, const ph_track_opts *opts,
                     double *x_end, int8_t *status, int8_t *reason, int32_t *steps,
                     ph_track_report *rep, void *stream);

/*
 * ph_track_batch -- many homotopies in one launch: the paths of nsys target
 * systems (total-degree start systems, roots-of-unity start points) are
 * concatenated into one device work queue; system s owns global path indices
 * path_off[s] .. path_off[s+1]-1.
 *   targets  : host array of nsys handles (square, n <= 32)
 *   gammas   : host [nsys][2]
 *   path_off : host int64[nsys + 1], path_off[0] = 0
 *   path_ids : host int64[path_off[nsys]] multi-index numbers of the tracked
 *              start solutions of each system, or NULL (0 .. npaths_s - 1);
 *              PH_EINVAL for a number outside 0 .. Bezout number - 1 (or,
 *              without path_ids, for more paths than start solutions)
 *   x_end, status, reason, steps : indexed by the global path index (ld >= total)
 * A path takes the next power of two >= its system's n lanes (4, 8, 16 or
 * 32); systems of one lane count share a work queue and a range of
 * workgroups sized by their share of the work.
 * Same synchrony, scratch and errors as ph_track.
 */
int ph_track_batch(int32_t nsys, const ph_system *const *targets, const double *gammas,
                   const int64_t *path_off, const int64_t *path_ids, const ph_track_opts *opts,
                   double *x_end, int64_t ld, int8_t *status, int8_t *reason, int32_t *steps,
                   ph_track_report *rep, void *stream);

/*
 * ph_track_autotune -- choose the launch shape of ph_track_batch (and of
 * ph_track with a total-degree start) for this batch: tracks a sample of
 * about `sample` paths (each system's first ones, in proportion to its path
 * count) under each candidate (schedule; for the graph schedule a fixed
 * rounds_per_launch of 8, 32 or 128 or a launch_ms of 1, 2 or 4; blocks_per_cu;
 * lanes_per_path: the natural count, twice or four times it) and writes *opts
 * with the fastest into *tuned (every other field copied).
 * With PH_AUTOTUNE_CACHE naming a file, a previous choice for the same
 * systems, path counts, prec and mixed is read from it instead of timing, and
 * a new choice is appended.  best_seconds (nullable) receives the sample's
 * time under the choice (0 when read from the file).  Allocates and frees
 * its own device outputs; synchronous.  Errors as ph_track_batch.
 */
int ph_track_autotune(int32_t nsys, const ph_system *const *targets, const double *gammas,
                      const int64_t *path_off, const int64_t *path_ids,
                      const ph_track_opts *opts, int64_t sample, ph_track_opts *tuned,
                      double *best_seconds, void *stream);

/* Message of the last failure on the calling thread ("" if none). */
const char *ph_last_error(void);

/*
 * ph_arith_probe -- apply one device arithmetic operation elementwise, for
 * checking the double double / quad double building blocks against exact
 * results.  op 0 add, 1 sub, 2 mul on reals [n][prec]; op 3 add, 4 multiply
 * on complexes [n][2][prec]; op 5 complex a times the real double b[i][0][0].
 * a, b, out: device arrays.  Asynchronous on stream.  PH_EINVAL on bad op/prec.
 */
int ph_arith_probe(int32_t prec, int32_t op, int64_t n, const double *a, const double *b,
                   double *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PH_H */
