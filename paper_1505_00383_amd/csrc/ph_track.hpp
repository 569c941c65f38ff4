// ph_track.hpp -- device-side descriptors of the path tracker.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/ph.h"

namespace ph {

// One system of a (possibly heterogeneous) batch.
struct SysDesc {
    const int32_t *eq_off;   // merged term table: target terms, then start terms
    const int4 *tdesc;
    const uint32_t *fac;
    const uint32_t *fac8;    // [term][8] factor words by term index
    const double *coef;
    const int64_t *path_ids; // multi-index number of every tracked path, or NULL (0..npaths-1)
    int64_t path_off;        // first global path index of this system (outputs)
    int64_t npaths;
    int64_t qoff;            // first queue index of this system inside its class
    double gre, gim;         // gamma
    int32_t n;               // equations = unknowns
    int32_t kmax;
    int32_t deg[64];         // degrees of the total-degree start system
    int64_t radix[64];       // mixed-radix place values prod_{l<i} deg[l]
};

// One lane-count class of a launch: systems sys_first..sys_end-1 of the
// descriptor table, whose paths are handed out by their own queue to the
// blocks below block_end (and at or above the previous class's block_end).
struct TrackClass {
    int np;
    int sys_first, sys_end;
    int block_end;
    int64_t total;
    unsigned long long *queue;
};

struct TrackArgs {
    const SysDesc *sys;
    int nsys;
    TrackClass cls[4];
    const double *x_start;   // SoA start points (rows (i*2+c)*L+l) or NULL: roots of unity
    int64_t ld_start;
    double *x_end;
    int64_t ld_end;
    int8_t *status;
    int8_t *reason;
    int32_t *steps;
    unsigned long long *stats;  // [0] steps [1] rejected [2] newton iterations [3 + reason] counts
    unsigned int *active;       // round schedule: waves still active after a launch
    void *state;                // round schedule: per-lane slot state
    double *hist;               // predictor orders 2..4: three older points per lane slot,
    int64_t hist_ld;            //   rows [q][re,im][limb], hist_ld = lane slots of the launch
    int rounds;                 // round schedule: rounds per launch
    unsigned long long budget;  // round schedule: wall-clock ticks per launch (0: rounds only)
    ph_track_opts o;
    double polish_tol;
    double eps_sing;
};

// occ == nullptr: launch the tracker kernel; else store the number of its
// workgroups that fit one CU at once (registers, LDS) and launch nothing.
int track_launch(const TrackArgs &a, int prec, int kmax, int blocks, size_t lds, hipStream_t st,
                 int *occ = nullptr);
// Per (residual limbs L, FP64 solves) launchers and slot-state helpers,
// instantiated in track_unit.hip.
template <int L, bool MIXED>
int track_launch_t(const TrackArgs &a, int kmax, int blocks, size_t lds, hipStream_t st, int *occ);
template <int L>
size_t slot_bytes_t();
template <int L>
int slot_init_launch_t(void *state, int64_t nslots, hipStream_t st);
size_t track_lds_bytes(int prec, int mixed, int np_max);
size_t slot_bytes(int prec);
int slot_init_launch(int prec, void *state, int64_t nslots, hipStream_t st);
int clear_counter_launch(unsigned int *c, hipStream_t st);

}  // namespace ph
