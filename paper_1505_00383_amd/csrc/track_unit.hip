// track_unit.hip -- launchers of the tracker kernel for one residual
// precision L (1, 2, 4) and one solve precision (MIXED: FP64 Newton solves;
// plain: L-limb solves).  The build compiles this file once per (L, MIXED)
// with -DPH_TRACK_L=<L> -DPH_TRACK_MIXED=<0|1>, so the six heavy kernel
// families compile in parallel; without those macros it instantiates all six.
#include "ph_track_dev.hpp"

namespace ph {

// occ == nullptr: launch; else store in *occ how many workgroups of the
// kernel that would be launched fit one CU at once, and launch nothing
template <int L, bool MIXED, int KMAX, int NPSEL>
static int launch_k(const TrackArgs &a, int blocks, size_t lds, hipStream_t st, int *occ)
{
    if (occ) {
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, track_kernel<L, KMAX, MIXED, NPSEL>, 64, lds);
        if (e != hipSuccess) return hip_fail(e, "track kernel occupancy");
        return PH_OK;
    }
    hipLaunchKernelGGL((track_kernel<L, KMAX, MIXED, NPSEL>), dim3(blocks), dim3(64), lds, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "track kernel launch");
    return PH_OK;
}

// several lane-count classes up to NPMAX in one launch
template <int L, bool MIXED, int NPMAX>
static int launch_n(const TrackArgs &a, int kmax, int blocks, size_t lds, hipStream_t st, int *occ)
{
    if (kmax <= 4) return launch_k<L, MIXED, 4, NPMAX>(a, blocks, lds, st, occ);
    return launch_k<L, MIXED, 8, NPMAX>(a, blocks, lds, st, occ);
}

// a single lane-count class NP: only its code, and a tighter term bound
template <int L, bool MIXED, int NP>
static int launch_1(const TrackArgs &a, int kmax, int blocks, size_t lds, hipStream_t st, int *occ)
{
    if (kmax <= 2) return launch_k<L, MIXED, 2, -NP>(a, blocks, lds, st, occ);
    if (kmax <= 4) return launch_k<L, MIXED, 4, -NP>(a, blocks, lds, st, occ);
    return launch_k<L, MIXED, 8, -NP>(a, blocks, lds, st, occ);
}

template <int L, bool MIXED>
int track_launch_t(const TrackArgs &a, int kmax, int blocks, size_t lds, hipStream_t st, int *occ)
{
    int npmax = 4, classes = 0;
    for (int c = 0; c < 4; ++c)
        if (a.cls[c].total > 0) {
            npmax = a.cls[c].np;
            ++classes;
        }
    if (classes == 1) {
        switch (npmax) {
        case 4: return launch_1<L, MIXED, 4>(a, kmax, blocks, lds, st, occ);
        case 8: return launch_1<L, MIXED, 8>(a, kmax, blocks, lds, st, occ);
        case 16: return launch_1<L, MIXED, 16>(a, kmax, blocks, lds, st, occ);
        default: return launch_1<L, MIXED, 32>(a, kmax, blocks, lds, st, occ);
        }
    }
    if (npmax <= 8) return launch_n<L, MIXED, 8>(a, kmax, blocks, lds, st, occ);
    if (npmax <= 16) return launch_n<L, MIXED, 16>(a, kmax, blocks, lds, st, occ);
    return launch_n<L, MIXED, 32>(a, kmax, blocks, lds, st, occ);
}

template <int L>
size_t slot_bytes_t()
{
    return sizeof(Slot<L>);
}

template <int L>
int slot_init_launch_t(void *state, int64_t nslots, hipStream_t st)
{
    dim3 grid((unsigned)((nslots + 255) / 256));
    hipLaunchKernelGGL(slot_init_kernel<L>, grid, dim3(256), 0, st, state, nslots);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "slot_init_kernel launch");
    return PH_OK;
}

#define PH_TRACK_INSTANTIATE(L_, M_)                                                             \
    template int track_launch_t<L_, M_>(const TrackArgs &, int, int, size_t, hipStream_t, int *);

#define PH_SLOT_INSTANTIATE(L_)                                                                  \
    template size_t slot_bytes_t<L_>();                                                          \
    template int slot_init_launch_t<L_>(void *, int64_t, hipStream_t);

#if defined(PH_TRACK_L) && defined(PH_TRACK_MIXED)
PH_TRACK_INSTANTIATE(PH_TRACK_L, (PH_TRACK_MIXED != 0))
#if PH_TRACK_MIXED
PH_SLOT_INSTANTIATE(PH_TRACK_L)
#endif
#else
PH_TRACK_INSTANTIATE(1, true)
PH_TRACK_INSTANTIATE(2, true)
PH_TRACK_INSTANTIATE(4, true)
PH_TRACK_INSTANTIATE(1, false)
PH_TRACK_INSTANTIATE(2, false)
PH_TRACK_INSTANTIATE(4, false)
PH_SLOT_INSTANTIATE(1)
PH_SLOT_INSTANTIATE(2)
PH_SLOT_INSTANTIATE(4)
#endif

}  // namespace ph
