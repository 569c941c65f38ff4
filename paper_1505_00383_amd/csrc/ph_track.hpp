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
    const double *coef;
    const int64_t *path_ids; // multi-index number of every tracked path, or NULL (0..npaths-1)
    int64_t path_off;        // first global path index of this system
    int64_t npaths;
    double gre, gim;         // gamma
    int32_t n;               // equations = unknowns
    int32_t kmax;
    int32_t deg[64];         // degrees of the total-degree start system
    int64_t radix[64];       // mixed-radix place values prod_{l<i} deg[l]
};

struct TrackArgs {
    const SysDesc *sys;
    int nsys;
    int64_t total_paths;
    const double *x_start;   // SoA start points (rows (i*2+c)*L+l) or NULL: roots of unity
    int64_t ld_start;
    double *x_end;
    int64_t ld_end;
    int8_t *status;
    int8_t *reason;
    int32_t *steps;
    int32_t *newton;
    unsigned long long *queue;  // next path to hand out
    unsigned long long *stats;  // [0] steps [1] rejected [2] newton iterations [3 + reason] counts
    ph_track_opts o;
    double polish_tol;
    double eps_sing;
};

int track_launch(const TrackArgs &a, int prec, int np, int kmax, int blocks, hipStream_t st);
int track_max_blocks(int prec, int np, int kmax, int mixed, int *blocks);

}  // namespace ph
