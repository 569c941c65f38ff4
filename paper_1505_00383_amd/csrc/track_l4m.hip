// track_l4m.hip -- tracker kernels, 4-limb residuals, FP64 (mixed) solves.
#include "ph_track_dev.hpp"

namespace ph {

template <int KMAX, int NPSEL>
static int launch_k(const TrackArgs &a, int blocks, size_t lds, hipStream_t st)
{
    hipLaunchKernelGGL((track_kernel<4, KMAX, true, NPSEL>), dim3(blocks), dim3(64), lds, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "track kernel launch");
    return PH_OK;
}

// several lane-count classes up to NPMAX in one launch
template <int NPMAX>
static int launch_n(const TrackArgs &a, int kmax, int blocks, size_t lds, hipStream_t st)
{
    if (kmax <= 4) return launch_k<4, NPMAX>(a, blocks, lds, st);
    return launch_k<8, NPMAX>(a, blocks, lds, st);
}

// a single lane-count class NP: only its code, and a tighter term bound
template <int NP>
static int launch_1(const TrackArgs &a, int kmax, int blocks, size_t lds, hipStream_t st)
{
    if (kmax <= 2) return launch_k<2, -NP>(a, blocks, lds, st);
    if (kmax <= 4) return launch_k<4, -NP>(a, blocks, lds, st);
    return launch_k<8, -NP>(a, blocks, lds, st);
}

int track_launch_l4m(const TrackArgs &a, int kmax, int blocks, size_t lds, hipStream_t st)
{
    int npmax = 4, classes = 0;
    for (int c = 0; c < 4; ++c)
        if (a.cls[c].total > 0) {
            npmax = a.cls[c].np;
            ++classes;
        }
    if (classes == 1) {
        switch (npmax) {
        case 4: return launch_1<4>(a, kmax, blocks, lds, st);
        case 8: return launch_1<8>(a, kmax, blocks, lds, st);
        case 16: return launch_1<16>(a, kmax, blocks, lds, st);
        default: return launch_1<32>(a, kmax, blocks, lds, st);
        }
    }
    if (npmax <= 8) return launch_n<8>(a, kmax, blocks, lds, st);
    if (npmax <= 16) return launch_n<16>(a, kmax, blocks, lds, st);
    return launch_n<32>(a, kmax, blocks, lds, st);
}

size_t slot_bytes_l4() { return sizeof(Slot<4>); }

int slot_init_launch_l4(void *state, int64_t nslots, hipStream_t st)
{
    dim3 grid((unsigned)((nslots + 255) / 256));
    hipLaunchKernelGGL(slot_init_kernel<4>, grid, dim3(256), 0, st, state, nslots);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "slot_init_kernel launch");
    return PH_OK;
}

}  // namespace ph
