// ph_internal.hpp -- internal structures shared by the system compiler, the
// evaluation kernels and the tracker.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ph.h"
#include "ph_sweep.hpp"

namespace ph {

// Error reporting: the message of the last failure on this thread.
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

#define PH_HIP(call)                                     \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return ph::hip_fail(e_, #call); \
    } while (0)


// Term descriptor: {k = number of factors, offset of the first factor word,
// sel = 0 for a target term (coefficient scaled by t) or 1 for a start-system
// term (scaled by gamma (1 - t)), unused}.
//
// One "homotopy table" is the merged term stream of target and start system,
// equation by equation: the instruction stream that every lane of a wave runs
// on its own point (Section 3: all threads of a block evaluate the same
// monomial at different points).
// Term record of the complex-double fast path: everything one term needs in
// one 192-byte block read through scalar loads, each field ready to use so
// that the kernel spends no scalar instructions decoding it: per factor l the
// LDS byte offsets of x_{j_l} and of x_{j_l}^{a_l - 1} (powers x, x^2, x^3
// and a row of ones are staged per point), the register index 2 j_l of its
// Jacobian column, and the exponent a_l as a double (folded into the FMA that
// accumulates the partial).
// Fast-path record groups: (k, m) with 0 <= m <= k <= 8, numbered k(k+1)/2 + m;
// DRUN offsets per equation (45 groups and the end).
constexpr int DRUN = 46;
inline constexpr int drun_group(int k, int m) { return k * (k + 1) / 2 + m; }

struct DTerm {
    double cre, cim;
    int32_t k;
    int32_t sel;     // bit 0: start term; bits 8..11: factors with a >= 3; 16..19: with a >= 2
    uint32_t xo[8];  // LDS byte offset of the factor's coordinate x_v (v * 1024)
    uint32_t po[8];  // LDS byte offset of x_v^(a-1), or of the ones row for a = 1
    uint32_t j2[8];  // 2 * v: register index of column v in the pinned row
    double a[8];     // exponents
    int32_t pad[2];
};

// Term record of the double-double and quad-double fast paths, in the same
// order as the DTerm records (the same d_run groups index both): the
// coefficient in all its limbs, per factor the LDS byte offsets of x_{j_l}
// and x_{j_l}^{a_l - 1} (both staging layouts give a (plane, variable) block
// 2048 bytes: DD four rows of 64 points, QD eight rows of 32 points), the
// accumulation-register index 8 j_l of its Jacobian column, and the exponent
// as a double.
struct MTerm {
    double c[8];     // [re, im][4 limbs]
    int32_t k, sel;  // as in DTerm
    uint32_t xo[8];
    uint32_t po[8];
    uint32_t jo[8];
    double a[8];
    int32_t pad[6];
};
static_assert(sizeof(MTerm) == 256, "MTerm is one 256-byte record");

struct DevTable {
    int n_eq = 0, n_var = 0, kmax = 0;
    int emax = 0;                // largest exponent of a target/start term
    bool dfast = false;          // the fast-path records below are valid
    int dfast_planes = 0;        // power planes staged in LDS (x, x^2, x^3)
    int32_t *d_eq_off = nullptr; // [n_eq + 1] offsets into dterm
    DTerm *dterm = nullptr;      // fast-path records (target terms, custom start terms)
    int32_t *d_deg = nullptr;    // [n_eq] total-degree start exponents (0: explicit start)
    bool mfast = false;          // the DD / QD records below are valid (LDS fits)
    MTerm *mterm = nullptr;      // DD / QD fast-path records, parallel to dterm
    int32_t *d_run = nullptr;    // [n_eq][DRUN]: records of equation i in group g (k
                                 // factors, m of them with a >= 2; g = drun_group(k, m))
                                 // are d_run[i*DRUN+g] .. d_run[i*DRUN+g+1]-1
    int64_t n_terms = 0, n_fac = 0;
    int32_t *eq_off = nullptr;   // [n_eq + 1]
    int4 *tdesc = nullptr;       // [n_terms]
    uint32_t *fac = nullptr;     // [n_fac]
    uint32_t *fac8 = nullptr;    // [n_terms][8]: each term's factor words, zero padded (tracker)
    double *coef = nullptr;      // [n_terms][2][4] limbs
    int32_t *zc_off = nullptr;   // [n_eq + 1] columns of each row no term touches
    int32_t *zc = nullptr;
    // the paper's unfused three-kernel design (coeff, mon, sum; an ablation):
    int64_t u_slots = 0;         // monomial slots: value and k partials per term
    int32_t *u_slot = nullptr;   // [n_terms] first slot of each term
    int32_t *u_off = nullptr;    // [n_eq * (1 + n_var) + 1] slots summed into each output
    int32_t *u_list = nullptr;   //   entry: H_i (entries 0..n_eq-1), then J_ij row-major
    void *block = nullptr;       // single device allocation holding all of the above
    void *u_scratch = nullptr;   // grow-only intermediate arrays of the unfused design,
    size_t u_scratch_bytes = 0;  //   sized by ph_eval_prepare (never by an evaluation)
};

// Kernel choice and tiling of one evaluation: kernel 0 automatic, 1 general
// (Jacobian row accumulated in the output), 2 register row (double, n <= 32),
// 3 fast path with the row pinned in registers (double: upper architectural
// registers; double double and quad double: accumulation registers), 4 the double fast path
// with a compiler-held row, 5 the unfused coeff / mon / sum kernels; W waves
// per workgroup, G equation groups (0: default).
struct EvalCfg {
    int kernel = 0, W = 0, G = 0;
};

struct HostSystem {
    uint64_t fingerprint = 0;  // FNV-1a of the defining arrays
    int n_eq = 0, n_var = 0, max_k = 0;
    std::vector<int32_t> eq_term_off, term_fac_off, fac_var, fac_exp, deg;
    std::vector<double> coef;  // [T][2][4]
};

struct ph_system_impl;

}  // namespace ph

struct ph_system {
    ph::HostSystem h;
    ph::DevTable total;  // target merged with the total-degree start system
    std::mutex mu;
    std::map<const ph_system *, ph::DevTable> with_start;  // custom start systems
    std::map<std::pair<const ph_system *, int>, ph::EvalCfg> eval_cfg;  // (start, prec) -> config
    // entries of the PH_AUTOTUNE_CACHE file for this target, read once when
    // the handle is created: (start fingerprint or 0, prec) -> config
    std::map<std::pair<uint64_t, int>, ph::EvalCfg> file_cfg;
    int device = 0;
};

namespace ph {
// Build and upload the merged table of (f, g); g == nullptr selects the
// total-degree start system g_i = x_i^{d_i} - 1.
int build_table(const HostSystem &f, const HostSystem *g, DevTable &out);
void free_table(DevTable &t);
// Table for (target, start), built on first use and cached in the target
// (allocates and synchronises when it builds).
int get_table(const ph_system *target, const ph_system *start, const DevTable **out);
// The same without building: PH_EINVAL when (target, start) was not prepared.
int find_table(const ph_system *target, const ph_system *start, const DevTable **out);
// Size the unfused design's intermediate arrays for npts points of prec limbs
// (grow-only; synchronises the device before releasing a smaller buffer).
int prepare_unfused(const ph_system *target, DevTable &tab, int prec, int64_t npts);
// Entries of the PH_AUTOTUNE_CACHE file for this target (called at creation).
void load_eval_cache(ph_system *s);
// The unfused three-kernel evaluation (kernel choice 5).
int unfused_launch(const DevTable &tab, const double gamma[2], int prec, int64_t npts,
                   const double *t, const double *x, int64_t ld, double *val, double *jac,
                   hipStream_t st);
// Double-double fast path (kernel choice 3 at prec 2): Jacobian row in the
// accumulation registers, W <= 4 waves per workgroup, G equation groups.
int dd_fast_launch(const DevTable &tab, const double gamma[2], int64_t npts, const double *t,
                   const double *x, int64_t ld, double *val, double *jac, int W, int G,
                   hipStream_t st);
// Quad-double fast path (kernel choice 3 at prec 4): two lanes per point, each
// lane's component of the Jacobian row in the accumulation registers.
int qd_fast_launch(const DevTable &tab, const double gamma[2], int64_t npts, const double *t,
                   const double *x, int64_t ld, double *val, double *jac, int W, int G,
                   hipStream_t st);
// Evaluation launch with an explicit configuration (cfg == NULL: defaults).
int eval_launch(const DevTable &tab, const double gamma[2], int prec, int64_t npts,
                const double *t, const double *x, int64_t ld, double *val, double *jac,
                hipStream_t st, const EvalCfg *cfg);
}  // namespace ph
