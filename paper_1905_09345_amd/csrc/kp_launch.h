// Host-side launchers of the kernels in kp_kernels.hip (internal to libkp).
#pragma once
#include <hip/hip_runtime.h>
#include "kp_device.h"

namespace kp {

struct LaunchCfg {
    int waves;      // waves of 64 lanes per workgroup of the assignment kernels
    int grid_cap;   // upper bound on workgroups of grid-stride kernels
    int depth;      // centroid chunks in flight per workgroup (BF16 mode): 1 or 3
};

// Per-point BF16 shadow and norms, initial centroid rows, drift rings at t=0.
hipError_t launch_prep(const ProbDev &P, hipStream_t s, const float *init_dev);
// Stages of one iteration, in launch order.
enum Stage { ST_BEGIN = 0, ST_FILTER, ST_SORT, ST_ASSIGN_DENSE, ST_ASSIGN, ST_RECHECK, ST_UPDATE, ST_CENTROIDS, ST_COUNT };
const char *stage_name(Stage st);
// The stages of a dense (first) or filtered iteration of problem P, in order.
int iteration_stages(const ProbDev &P, bool dense, Stage out[ST_COUNT]);
// Launch the kernels of one stage.
hipError_t launch_stage(const ProbDev &P, hipStream_t s, Stage st, bool dense, const LaunchCfg &cfg);
// One K-means iteration (dense = every distance) of one problem.
hipError_t launch_iteration(const ProbDev &P, hipStream_t s, bool dense, const LaunchCfg &cfg);
// Current assignment as original centroid indices.
hipError_t launch_labels(const ProbDev &P, hipStream_t s, int *out);
// Current centroids in original order (either output may be null).
hipError_t launch_centroids_out(const ProbDev &P, hipStream_t s, float *c32, double *c64);

}  // namespace kp
