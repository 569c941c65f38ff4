// probe.hip -- element-wise access to the device multi-limb arithmetic, so the
// double double / quad double building blocks can be checked against exact
// rational results.
#include <hip/hip_runtime.h>

#include "ph_arith.hpp"
#include "ph_internal.hpp"

namespace ph {

template <int L>
__global__ void __launch_bounds__(256) probe_kernel(int op, int64_t n, const double *__restrict__ a,
                                                    const double *__restrict__ b,
                                                    double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (op < 3) {  // real ops on [n][L]
        R<L> x, y;
#pragma unroll
        for (int l = 0; l < L; ++l) {
            x.v[l] = a[i * L + l];
            y.v[l] = b[i * L + l];
        }
        R<L> r = op == 0 ? r_add<L>(x, y) : (op == 1 ? r_sub<L>(x, y) : r_mul<L>(x, y));
#pragma unroll
        for (int l = 0; l < L; ++l) out[i * L + l] = r.v[l];
    } else {  // complex ops on [n][2][L]
        C<L> x, y;
#pragma unroll
        for (int l = 0; l < L; ++l) {
            x.re.v[l] = a[(i * 2) * L + l];
            x.im.v[l] = a[(i * 2 + 1) * L + l];
            y.re.v[l] = b[(i * 2) * L + l];
            y.im.v[l] = b[(i * 2 + 1) * L + l];
        }
        C<L> r;
        if (op == 3)
            r = c_add<L>(x, y);
        else if (op == 4)
            r = c_mul<L>(x, y);
        else
            r = c_mul_d<L>(x, y.re.v[0]);
#pragma unroll
        for (int l = 0; l < L; ++l) {
            out[(i * 2) * L + l] = r.re.v[l];
            out[(i * 2 + 1) * L + l] = r.im.v[l];
        }
    }
}

}  // namespace ph

using namespace ph;

extern "C" int ph_arith_probe(int32_t prec, int32_t op, int64_t n, const double *a, const double *b,
                              double *out, void *stream)
{
    if (prec != 1 && prec != 2 && prec != 4) return fail(PH_EINVAL, "prec must be 1, 2 or 4");
    if (op < 0 || op > 5) return fail(PH_EINVAL, "op must be in 0..5");
    if (n < 0) return fail(PH_EINVAL, "n < 0");
    if (n == 0) return PH_OK;
    if (!a || !b || !out) return fail(PH_EINVAL, "null pointer");
    hipStream_t st = (hipStream_t)stream;
    dim3 grid((unsigned)((n + 255) / 256));
    switch (prec) {
    case 1: hipLaunchKernelGGL(probe_kernel<1>, grid, dim3(256), 0, st, op, n, a, b, out); break;
    case 2: hipLaunchKernelGGL(probe_kernel<2>, grid, dim3(256), 0, st, op, n, a, b, out); break;
    default: hipLaunchKernelGGL(probe_kernel<4>, grid, dim3(256), 0, st, op, n, a, b, out); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "probe_kernel launch");
    return PH_OK;
}
