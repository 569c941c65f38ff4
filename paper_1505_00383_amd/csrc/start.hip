// start.hip -- start solutions of the total-degree start system
// g_i = x_i^{d_i} - 1 of the homotopy of Eq. (1): roots of unity, path index
// to multi-index by little-endian mixed radix.
#include <hip/hip_runtime.h>

#include "ph_arith.hpp"
#include "ph_internal.hpp"

namespace ph {

// sqrt(3)/2 in L limbs: y ~ 1/sqrt(3) by Newton's iteration
// y <- y + y (1 - 3 y^2) / 2 from the FP64 seed (53 -> 106 -> 212 bits), then
// s = 3 y corrected once by s <- s + y (3 - s^2) / 2, then halved (exact).
template <int L>
__device__ R<L> half_sqrt3()
{
    if constexpr (L == 1) {
        return r_from<1>(0.5 * sqrt(3.0));
    } else {
        R<L> y = r_from<L>(1.0 / sqrt(3.0));
        const R<L> three = r_from<L>(3.0);
        const int steps = L == 2 ? 2 : 3;
        for (int s = 0; s < steps; ++s) {
            R<L> r = r_sub<L>(r_from<L>(1.0), r_mul<L>(three, r_mul<L>(y, y)));
            y = r_add<L>(y, r_mul_d<L>(r_mul<L>(y, r), 0.5));
        }
        R<L> s = r_mul<L>(three, y);
        R<L> r = r_sub<L>(three, r_mul<L>(s, s));
        s = r_add<L>(s, r_mul_d<L>(r_mul<L>(y, r), 0.5));
        return r_mul_d<L>(s, 0.5);
    }
}

struct DegArg {
    int32_t d[64];
};

template <int L>
__global__ void __launch_bounds__(256) start_kernel(DegArg deg, int n,
                                                    int64_t first, int64_t npaths,
                                                    double *__restrict__ x, int64_t ld)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npaths) return;
    const R<L> h3 = half_sqrt3<L>();
    int64_t p = first + q;
    for (int i = 0; i < n; ++i) {
        const int d = deg.d[i];
        const int k = (int)(p % d);
        p /= d;
        const int a = ((12 / d) * k) % 12;  // angle 2 pi k / d in units of 30 degrees
        R<L> c = r_zero<L>(), s = r_zero<L>();
        switch (a) {
        case 0: c = r_from<L>(1.0); break;
        case 2: c = r_from<L>(0.5); s = h3; break;
        case 3: s = r_from<L>(1.0); break;
        case 4: c = r_from<L>(-0.5); s = h3; break;
        case 6: c = r_from<L>(-1.0); break;
        case 8: c = r_from<L>(-0.5); s = r_neg<L>(h3); break;
        case 9: s = r_from<L>(-1.0); break;
        case 10: c = r_from<L>(0.5); s = r_neg<L>(h3); break;
        default: break;
        }
#pragma unroll
        for (int l = 0; l < L; ++l) {
            x[((int64_t)(i * 2 + 0) * L + l) * ld + q] = c.v[l];
            x[((int64_t)(i * 2 + 1) * L + l) * ld + q] = s.v[l];
        }
    }
}

}  // namespace ph

using namespace ph;

extern "C" int ph_start_solutions(const ph_system *target, int32_t prec, int64_t first_path,
                                  int64_t npaths, double *x, int64_t ld, void *stream)
{
    if (!target) return fail(PH_EINVAL, "null target");
    if (prec != 1 && prec != 2 && prec != 4) return fail(PH_EINVAL, "prec must be 1, 2 or 4");
    if (npaths < 0 || first_path < 0) return fail(PH_EINVAL, "negative path range");
    if (npaths == 0) return PH_OK;
    if (!x || ld < npaths) return fail(PH_EINVAL, "null x or ld < npaths");
    const int n = target->h.n_var;
    if (target->h.n_eq != n) return fail(PH_EINVAL, "start solutions need a square system");
    for (int i = 0; i < n; ++i) {
        int d = target->h.deg[i];
        if (d < 1 || 12 % d != 0 || d == 12)
            return fail(PH_EUNSUPPORTED, "start solutions need every degree in {1,2,3,4,6}");
    }
    hipStream_t st = (hipStream_t)stream;
    DegArg ddeg;
    for (int i = 0; i < 64; ++i) ddeg.d[i] = i < n ? target->h.deg[i] : 1;
    dim3 grid((unsigned)((npaths + 255) / 256));
    switch (prec) {
    case 1: hipLaunchKernelGGL(start_kernel<1>, grid, dim3(256), 0, st, ddeg, n, first_path, npaths, x, ld); break;
    case 2: hipLaunchKernelGGL(start_kernel<2>, grid, dim3(256), 0, st, ddeg, n, first_path, npaths, x, ld); break;
    default: hipLaunchKernelGGL(start_kernel<4>, grid, dim3(256), 0, st, ddeg, n, first_path, npaths, x, ld); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "start_kernel launch");
    return PH_OK;
}
