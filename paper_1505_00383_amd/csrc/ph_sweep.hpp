// ph_sweep.hpp -- the reverse-mode evaluation of one term and its gradient
// (Section 1 decomposition, Section 3 Table 6), written once for every number
// type: the device's complex D/DD/QD, and any host type that provides
// num_mul(a, b) and num_scale(a, double) (the unit test instantiates it with a
// symbolic type to check the product sequence of Table 6).
//
// A term is c * prod_{l<k} x_{j_l}^{a_l}.  With the common factor
// cf = c * prod x_{j_l}^{a_l - 1}:
//   q_0 = cf, q_l = q_{l-1} * x_{j_{l-1}}      forward products (k - 1)
//   value = q_{k-1} * x_{j_{k-1}}              (1)
//   d/dx_{j_l} = a_l * q_l * s_{l+1},  s_{k-1} = x_{j_{k-1}},
//   s_l = s_{l+1} * x_{j_l}                    backward: (k - 1) cross + (k - 2) suffix
// 3k - 3 products in all, of which 3k - 5 form the bare variable product and
// its k partial products and two fold cf in (q_1 = cf x_{j_0}, and cf times
// the last suffix).  Powers of the common factor take sum (a_l - 1) products.
#pragma once

#include <cstdint>

#ifdef __HIPCC__
#define PH_SW __host__ __device__ __forceinline__
#else
#define PH_SW inline
#endif

namespace ph {

// Factor word of the term tables: variable in bits 0..15, exponent in bits
// 16..30, bit 31 set when this factor is the first contribution of its
// equation to that Jacobian column.
constexpr uint32_t FAC_FIRST = 0x80000000u;
PH_SW int fac_var(uint32_t w) { return int(w & 0xffffu); }
PH_SW int fac_exp(uint32_t w) { return int((w >> 16) & 0x7fffu); }

// X(var) loads a coordinate; P(l, word, partial) consumes the partial
// derivative with respect to factor l (already scaled by its exponent).
// Returns the value of the term.  k must be in 1..KMAX.  With KEEPX = false
// the coordinates are loaded again for the backward products instead of
// being held (fewer registers for wide number types).
template <int KMAX, bool JAC, bool KEEPX = true, class Num, class XF, class PF>
PH_SW Num term_sweep(int k, const uint32_t *fw, Num c, XF &&X, PF &&P)
{
    Num xv[KEEPX ? KMAX : 1];
    auto xat = [&](int l) -> Num {
        if constexpr (KEEPX)
            return xv[l];
        else
            return X(fac_var(fw[l]));
    };
    Num q[KMAX];
    Num cf = c;
#pragma unroll
    for (int l = 0; l < KMAX; ++l) {
        if (l < k) {
            const Num xl = X(fac_var(fw[l]));
            if constexpr (KEEPX) xv[l] = xl;
            const int e = fac_exp(fw[l]);
            for (int r = 1; r < e; ++r) cf = num_mul(cf, xl);
        }
    }
    q[0] = cf;
#pragma unroll
    for (int l = 1; l < KMAX; ++l)
        if (l < k) q[l] = num_mul(q[l - 1], xat(l - 1));
    // last forward product and last coordinate, selected with static indices
    Num last = q[0];
    Num xlast;
    if constexpr (KEEPX) xlast = xv[0];
    uint32_t wlast = fw[0];
#pragma unroll
    for (int l = 1; l < KMAX; ++l)
        if (l == k - 1) {
            last = q[l];
            wlast = fw[l];
            if constexpr (KEEPX) xlast = xv[l];
        }
    if constexpr (!KEEPX) xlast = X(fac_var(wlast));
    Num value = num_mul(last, xlast);
    if constexpr (JAC) {
        Num sfx = xlast;
#pragma unroll
        for (int l = KMAX - 1; l >= 0; --l) {
            if (l < k) {
                Num part = (l == k - 1) ? q[l] : num_mul(q[l], sfx);
                if (l < k - 1 && l > 0) sfx = num_mul(sfx, xat(l));
                const int e = fac_exp(fw[l]);
                if (e != 1) part = num_scale(part, (double)e);
                P(l, fw[l], part);
            }
        }
    }
    return value;
}

}  // namespace ph
