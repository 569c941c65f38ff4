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

#define PH_ACC_CLOBBERS "a0","a1","a2","a3","a4","a5","a6","a7","a8","a9","a10","a11","a12","a13","a14","a15","a16","a17","a18","a19","a20","a21","a22","a23","a24","a25","a26","a27","a28","a29","a30","a31","a32","a33","a34","a35","a36","a37","a38","a39","a40","a41","a42","a43","a44","a45","a46","a47","a48","a49","a50","a51","a52","a53","a54","a55","a56","a57","a58","a59","a60","a61","a62","a63","a64","a65","a66","a67","a68","a69","a70","a71","a72","a73","a74","a75","a76","a77","a78","a79","a80","a81","a82","a83","a84","a85","a86","a87","a88","a89","a90","a91","a92","a93","a94","a95","a96","a97","a98","a99","a100","a101","a102","a103","a104","a105","a106","a107","a108","a109","a110","a111","a112","a113","a114","a115","a116","a117","a118","a119","a120","a121","a122","a123","a124","a125","a126","a127","a128","a129","a130","a131","a132","a133","a134","a135","a136","a137","a138","a139","a140","a141","a142","a143","a144","a145","a146","a147","a148","a149","a150","a151","a152","a153","a154","a155","a156","a157","a158","a159","a160","a161","a162","a163","a164","a165","a166","a167","a168","a169","a170","a171","a172","a173","a174","a175","a176","a177","a178","a179","a180","a181","a182","a183","a184","a185","a186","a187","a188","a189","a190","a191","a192","a193","a194","a195","a196","a197","a198","a199","a200","a201","a202","a203","a204","a205","a206","a207","a208","a209","a210","a211","a212","a213","a214","a215","a216","a217","a218","a219","a220","a221","a222","a223","a224","a225","a226","a227","a228","a229","a230","a231","a232","a233","a234","a235","a236","a237","a238","a239","a240","a241","a242","a243","a244","a245","a246","a247","a248","a249","a250","a251","a252","a253","a254","a255"

// The Jacobian row in the accumulation registers.  Every statement that
// touches them lists all 256 as clobbered, so the compiler never keeps a value
// of its own there across a row access; the compiled kernel is checked to
// contain no compiler-generated instruction that names an AGPR or M0 (the
// index register of the GPR indexing mode).  Column offsets jo = 8 j with
// 0 <= j < 32 (the fast path requires n <= 32).
struct ARow {
    __device__ __forceinline__ void zero()
    {
        asm volatile("v_accvgpr_write_b32 a0, 0\n\tv_accvgpr_write_b32 a1, 0\n\tv_accvgpr_write_b32 a2, 0\n\tv_accvgpr_write_b32 a3, 0\n\tv_accvgpr_write_b32 a4, 0\n\tv_accvgpr_write_b32 a5, 0\n\tv_accvgpr_write_b32 a6, 0\n\tv_accvgpr_write_b32 a7, 0\n\tv_accvgpr_write_b32 a8, 0\n\tv_accvgpr_write_b32 a9, 0\n\tv_accvgpr_write_b32 a10, 0\n\tv_accvgpr_write_b32 a11, 0\n\tv_accvgpr_write_b32 a12, 0\n\tv_accvgpr_write_b32 a13, 0\n\tv_accvgpr_write_b32 a14, 0\n\tv_accvgpr_write_b32 a15, 0\n\tv_accvgpr_write_b32 a16, 0\n\tv_accvgpr_write_b32 a17, 0\n\tv_accvgpr_write_b32 a18, 0\n\tv_accvgpr_write_b32 a19, 0\n\tv_accvgpr_write_b32 a20, 0\n\tv_accvgpr_write_b32 a21, 0\n\tv_accvgpr_write_b32 a22, 0\n\tv_accvgpr_write_b32 a23, 0\n\tv_accvgpr_write_b32 a24, 0\n\tv_accvgpr_write_b32 a25, 0\n\tv_accvgpr_write_b32 a26, 0\n\tv_accvgpr_write_b32 a27, 0\n\tv_accvgpr_write_b32 a28, 0\n\tv_accvgpr_write_b32 a29, 0\n\tv_accvgpr_write_b32 a30, 0\n\tv_accvgpr_write_b32 a31, 0\n\tv_accvgpr_write_b32 a32, 0\n\tv_accvgpr_write_b32 a33, 0\n\tv_accvgpr_write_b32 a34, 0\n\tv_accvgpr_write_b32 a35, 0\n\tv_accvgpr_write_b32 a36, 0\n\tv_accvgpr_write_b32 a37, 0\n\tv_accvgpr_write_b32 a38, 0\n\tv_accvgpr_write_b32 a39, 0\n\tv_accvgpr_write_b32 a40, 0\n\tv_accvgpr_write_b32 a41, 0\n\tv_accvgpr_write_b32 a42, 0\n\tv_accvgpr_write_b32 a43, 0\n\tv_accvgpr_write_b32 a44, 0\n\tv_accvgpr_write_b32 a45, 0\n\tv_accvgpr_write_b32 a46, 0\n\tv_accvgpr_write_b32 a47, 0\n\tv_accvgpr_write_b32 a48, 0\n\tv_accvgpr_write_b32 a49, 0\n\tv_accvgpr_write_b32 a50, 0\n\tv_accvgpr_write_b32 a51, 0\n\tv_accvgpr_write_b32 a52, 0\n\tv_accvgpr_write_b32 a53, 0\n\tv_accvgpr_write_b32 a54, 0\n\tv_accvgpr_write_b32 a55, 0\n\tv_accvgpr_write_b32 a56, 0\n\tv_accvgpr_write_b32 a57, 0\n\tv_accvgpr_write_b32 a58, 0\n\tv_accvgpr_write_b32 a59, 0\n\tv_accvgpr_write_b32 a60, 0\n\tv_accvgpr_write_b32 a61, 0\n\tv_accvgpr_write_b32 a62, 0\n\tv_accvgpr_write_b32 a63, 0\n\tv_accvgpr_write_b32 a64, 0\n\tv_accvgpr_write_b32 a65, 0\n\tv_accvgpr_write_b32 a66, 0\n\tv_accvgpr_write_b32 a67, 0\n\tv_accvgpr_write_b32 a68, 0\n\tv_accvgpr_write_b32 a69, 0\n\tv_accvgpr_write_b32 a70, 0\n\tv_accvgpr_write_b32 a71, 0\n\tv_accvgpr_write_b32 a72, 0\n\tv_accvgpr_write_b32 a73, 0\n\tv_accvgpr_write_b32 a74, 0\n\tv_accvgpr_write_b32 a75, 0\n\tv_accvgpr_write_b32 a76, 0\n\tv_accvgpr_write_b32 a77, 0\n\tv_accvgpr_write_b32 a78, 0\n\tv_accvgpr_write_b32 a79, 0\n\tv_accvgpr_write_b32 a80, 0\n\tv_accvgpr_write_b32 a81, 0\n\tv_accvgpr_write_b32 a82, 0\n\tv_accvgpr_write_b32 a83, 0\n\tv_accvgpr_write_b32 a84, 0\n\tv_accvgpr_write_b32 a85, 0\n\tv_accvgpr_write_b32 a86, 0\n\tv_accvgpr_write_b32 a87, 0\n\tv_accvgpr_write_b32 a88, 0\n\tv_accvgpr_write_b32 a89, 0\n\tv_accvgpr_write_b32 a90, 0\n\tv_accvgpr_write_b32 a91, 0\n\tv_accvgpr_write_b32 a92, 0\n\tv_accvgpr_write_b32 a93, 0\n\tv_accvgpr_write_b32 a94, 0\n\tv_accvgpr_write_b32 a95, 0\n\tv_accvgpr_write_b32 a96, 0\n\tv_accvgpr_write_b32 a97, 0\n\tv_accvgpr_write_b32 a98, 0\n\tv_accvgpr_write_b32 a99, 0\n\tv_accvgpr_write_b32 a100, 0\n\tv_accvgpr_write_b32 a101, 0\n\tv_accvgpr_write_b32 a102, 0\n\tv_accvgpr_write_b32 a103, 0\n\tv_accvgpr_write_b32 a104, 0\n\tv_accvgpr_write_b32 a105, 0\n\tv_accvgpr_write_b32 a106, 0\n\tv_accvgpr_write_b32 a107, 0\n\tv_accvgpr_write_b32 a108, 0\n\tv_accvgpr_write_b32 a109, 0\n\tv_accvgpr_write_b32 a110, 0\n\tv_accvgpr_write_b32 a111, 0\n\tv_accvgpr_write_b32 a112, 0\n\tv_accvgpr_write_b32 a113, 0\n\tv_accvgpr_write_b32 a114, 0\n\tv_accvgpr_write_b32 a115, 0\n\tv_accvgpr_write_b32 a116, 0\n\tv_accvgpr_write_b32 a117, 0\n\tv_accvgpr_write_b32 a118, 0\n\tv_accvgpr_write_b32 a119, 0\n\tv_accvgpr_write_b32 a120, 0\n\tv_accvgpr_write_b32 a121, 0\n\tv_accvgpr_write_b32 a122, 0\n\tv_accvgpr_write_b32 a123, 0\n\tv_accvgpr_write_b32 a124, 0\n\tv_accvgpr_write_b32 a125, 0\n\tv_accvgpr_write_b32 a126, 0\n\tv_accvgpr_write_b32 a127, 0\n\tv_accvgpr_write_b32 a128, 0\n\tv_accvgpr_write_b32 a129, 0\n\tv_accvgpr_write_b32 a130, 0\n\tv_accvgpr_write_b32 a131, 0\n\tv_accvgpr_write_b32 a132, 0\n\tv_accvgpr_write_b32 a133, 0\n\tv_accvgpr_write_b32 a134, 0\n\tv_accvgpr_write_b32 a135, 0\n\tv_accvgpr_write_b32 a136, 0\n\tv_accvgpr_write_b32 a137, 0\n\tv_accvgpr_write_b32 a138, 0\n\tv_accvgpr_write_b32 a139, 0\n\tv_accvgpr_write_b32 a140, 0\n\tv_accvgpr_write_b32 a141, 0\n\tv_accvgpr_write_b32 a142, 0\n\tv_accvgpr_write_b32 a143, 0\n\tv_accvgpr_write_b32 a144, 0\n\tv_accvgpr_write_b32 a145, 0\n\tv_accvgpr_write_b32 a146, 0\n\tv_accvgpr_write_b32 a147, 0\n\tv_accvgpr_write_b32 a148, 0\n\tv_accvgpr_write_b32 a149, 0\n\tv_accvgpr_write_b32 a150, 0\n\tv_accvgpr_write_b32 a151, 0\n\tv_accvgpr_write_b32 a152, 0\n\tv_accvgpr_write_b32 a153, 0\n\tv_accvgpr_write_b32 a154, 0\n\tv_accvgpr_write_b32 a155, 0\n\tv_accvgpr_write_b32 a156, 0\n\tv_accvgpr_write_b32 a157, 0\n\tv_accvgpr_write_b32 a158, 0\n\tv_accvgpr_write_b32 a159, 0\n\tv_accvgpr_write_b32 a160, 0\n\tv_accvgpr_write_b32 a161, 0\n\tv_accvgpr_write_b32 a162, 0\n\tv_accvgpr_write_b32 a163, 0\n\tv_accvgpr_write_b32 a164, 0\n\tv_accvgpr_write_b32 a165, 0\n\tv_accvgpr_write_b32 a166, 0\n\tv_accvgpr_write_b32 a167, 0\n\tv_accvgpr_write_b32 a168, 0\n\tv_accvgpr_write_b32 a169, 0\n\tv_accvgpr_write_b32 a170, 0\n\tv_accvgpr_write_b32 a171, 0\n\tv_accvgpr_write_b32 a172, 0\n\tv_accvgpr_write_b32 a173, 0\n\tv_accvgpr_write_b32 a174, 0\n\tv_accvgpr_write_b32 a175, 0\n\tv_accvgpr_write_b32 a176, 0\n\tv_accvgpr_write_b32 a177, 0\n\tv_accvgpr_write_b32 a178, 0\n\tv_accvgpr_write_b32 a179, 0\n\tv_accvgpr_write_b32 a180, 0\n\tv_accvgpr_write_b32 a181, 0\n\tv_accvgpr_write_b32 a182, 0\n\tv_accvgpr_write_b32 a183, 0\n\tv_accvgpr_write_b32 a184, 0\n\tv_accvgpr_write_b32 a185, 0\n\tv_accvgpr_write_b32 a186, 0\n\tv_accvgpr_write_b32 a187, 0\n\tv_accvgpr_write_b32 a188, 0\n\tv_accvgpr_write_b32 a189, 0\n\tv_accvgpr_write_b32 a190, 0\n\tv_accvgpr_write_b32 a191, 0\n\tv_accvgpr_write_b32 a192, 0\n\tv_accvgpr_write_b32 a193, 0\n\tv_accvgpr_write_b32 a194, 0\n\tv_accvgpr_write_b32 a195, 0\n\tv_accvgpr_write_b32 a196, 0\n\tv_accvgpr_write_b32 a197, 0\n\tv_accvgpr_write_b32 a198, 0\n\tv_accvgpr_write_b32 a199, 0\n\tv_accvgpr_write_b32 a200, 0\n\tv_accvgpr_write_b32 a201, 0\n\tv_accvgpr_write_b32 a202, 0\n\tv_accvgpr_write_b32 a203, 0\n\tv_accvgpr_write_b32 a204, 0\n\tv_accvgpr_write_b32 a205, 0\n\tv_accvgpr_write_b32 a206, 0\n\tv_accvgpr_write_b32 a207, 0\n\tv_accvgpr_write_b32 a208, 0\n\tv_accvgpr_write_b32 a209, 0\n\tv_accvgpr_write_b32 a210, 0\n\tv_accvgpr_write_b32 a211, 0\n\tv_accvgpr_write_b32 a212, 0\n\tv_accvgpr_write_b32 a213, 0\n\tv_accvgpr_write_b32 a214, 0\n\tv_accvgpr_write_b32 a215, 0\n\tv_accvgpr_write_b32 a216, 0\n\tv_accvgpr_write_b32 a217, 0\n\tv_accvgpr_write_b32 a218, 0\n\tv_accvgpr_write_b32 a219, 0\n\tv_accvgpr_write_b32 a220, 0\n\tv_accvgpr_write_b32 a221, 0\n\tv_accvgpr_write_b32 a222, 0\n\tv_accvgpr_write_b32 a223, 0\n\tv_accvgpr_write_b32 a224, 0\n\tv_accvgpr_write_b32 a225, 0\n\tv_accvgpr_write_b32 a226, 0\n\tv_accvgpr_write_b32 a227, 0\n\tv_accvgpr_write_b32 a228, 0\n\tv_accvgpr_write_b32 a229, 0\n\tv_accvgpr_write_b32 a230, 0\n\tv_accvgpr_write_b32 a231, 0\n\tv_accvgpr_write_b32 a232, 0\n\tv_accvgpr_write_b32 a233, 0\n\tv_accvgpr_write_b32 a234, 0\n\tv_accvgpr_write_b32 a235, 0\n\tv_accvgpr_write_b32 a236, 0\n\tv_accvgpr_write_b32 a237, 0\n\tv_accvgpr_write_b32 a238, 0\n\tv_accvgpr_write_b32 a239, 0\n\tv_accvgpr_write_b32 a240, 0\n\tv_accvgpr_write_b32 a241, 0\n\tv_accvgpr_write_b32 a242, 0\n\tv_accvgpr_write_b32 a243, 0\n\tv_accvgpr_write_b32 a244, 0\n\tv_accvgpr_write_b32 a245, 0\n\tv_accvgpr_write_b32 a246, 0\n\tv_accvgpr_write_b32 a247, 0\n\tv_accvgpr_write_b32 a248, 0\n\tv_accvgpr_write_b32 a249, 0\n\tv_accvgpr_write_b32 a250, 0\n\tv_accvgpr_write_b32 a251, 0\n\tv_accvgpr_write_b32 a252, 0\n\tv_accvgpr_write_b32 a253, 0\n\tv_accvgpr_write_b32 a254, 0\n\tv_accvgpr_write_b32 a255, 0" ::: PH_ACC_CLOBBERS);
    }
    // the eight dwords of column jo / 8
    __device__ __forceinline__ void read(uint32_t jo, double &rh, double &rl, double &ih, double &il)
    {
        unsigned w0, w1, w2, w3, w4, w5, w6, w7;
        asm volatile("s_set_gpr_idx_on %8, gpr_idx(SRC0)\n\t"
                     "v_accvgpr_read_b32 %0, a0\n\t"
                     "v_accvgpr_read_b32 %1, a1\n\t"
                     "v_accvgpr_read_b32 %2, a2\n\t"
                     "v_accvgpr_read_b32 %3, a3\n\t"
                     "v_accvgpr_read_b32 %4, a4\n\t"
                     "v_accvgpr_read_b32 %5, a5\n\t"
                     "v_accvgpr_read_b32 %6, a6\n\t"
                     "v_accvgpr_read_b32 %7, a7\n\t"
                     "s_set_gpr_idx_off"
                     : "=v"(w0), "=v"(w1), "=v"(w2), "=v"(w3), "=v"(w4), "=v"(w5), "=v"(w6), "=v"(w7)
                     : "s"(jo)
                     : PH_ACC_CLOBBERS);
        rh = __builtin_bit_cast(double, ((unsigned long long)w1 << 32) | w0);
        rl = __builtin_bit_cast(double, ((unsigned long long)w3 << 32) | w2);
        ih = __builtin_bit_cast(double, ((unsigned long long)w5 << 32) | w4);
        il = __builtin_bit_cast(double, ((unsigned long long)w7 << 32) | w6);
    }
    __device__ __forceinline__ void write(uint32_t jo, double rh, double rl, double ih, double il)
    {
        const unsigned long long a = __builtin_bit_cast(unsigned long long, rh);
        const unsigned long long b = __builtin_bit_cast(unsigned long long, rl);
        const unsigned long long c = __builtin_bit_cast(unsigned long long, ih);
        const unsigned long long d = __builtin_bit_cast(unsigned long long, il);
        asm volatile("s_set_gpr_idx_on %8, gpr_idx(DST)\n\t"
                     "v_accvgpr_write_b32 a0, %0\n\t"
                     "v_accvgpr_write_b32 a1, %1\n\t"
                     "v_accvgpr_write_b32 a2, %2\n\t"
                     "v_accvgpr_write_b32 a3, %3\n\t"
                     "v_accvgpr_write_b32 a4, %4\n\t"
                     "v_accvgpr_write_b32 a5, %5\n\t"
                     "v_accvgpr_write_b32 a6, %6\n\t"
                     "v_accvgpr_write_b32 a7, %7\n\t"
                     "s_set_gpr_idx_off"
                     :
                     : "v"((unsigned)a), "v"((unsigned)(a >> 32)), "v"((unsigned)b), "v"((unsigned)(b >> 32)),
                       "v"((unsigned)c), "v"((unsigned)(c >> 32)), "v"((unsigned)d), "v"((unsigned)(d >> 32)),
                       "s"(jo)
                     : PH_ACC_CLOBBERS);
    }
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

struct MHead {
    double c[4];  // re hi, re lo, im hi, im lo
    int sel;
    uint32_t xo[8], po[8], jo[8];
    double a[8];
};

template <int K, int M>
__device__ __forceinline__ MHead mfast_head(const MTerm *__restrict__ r)
{
    MHead h;
    h.c[0] = r->c[0];
    h.c[1] = r->c[1];
    h.c[2] = r->c[4];
    h.c[3] = r->c[5];
    h.sel = r->sel;
#pragma unroll
    for (int l = 0; l < K; ++l) h.xo[l] = r->xo[l];
#pragma unroll
    for (int l = 0; l < M; ++l) h.po[l] = r->po[l];
#pragma unroll
    for (int l = 0; l < K; ++l) h.jo[l] = r->jo[l];
#pragma unroll
    for (int l = 0; l < K; ++l) h.a[l] = r->a[l];
    return h;
}

// One term with K factors, the first M of them with a >= 2 (same product
// order as the complex-double fast path).
template <int K, int M>
__device__ __forceinline__ void mfast_sweep(const MHead &h, const MTerm *__restrict__ rnext, MHead &hnext,
                                            const char *__restrict__ xb, int lane, C<2> cf, ARow &row,
                                            C<2> &v)
{
    C<2> xv[K], pw[M > 0 ? M : 1], sf[K];
#pragma unroll
    for (int l = 0; l < K; ++l) xv[l] = lds2(xb, h.xo[l], lane);
#pragma unroll
    for (int l = 0; l < M; ++l) pw[l] = lds2(xb, h.po[l], lane);
    hnext = mfast_head<K, M>(rnext);
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

__device__ __forceinline__ C<2> mcoef(const MHead &h, const C<2> &gs, double tv)
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
        MHead h = mfast_head<K, M>(mt + s0);
        for (int s = s0; s < s1; ++s) {
            const MTerm *rn = mt + (s + 1 < s1 ? s + 1 : s);
            MHead hn;
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
            MHead h = mfast_head<0, 0>(mterm + s);
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
