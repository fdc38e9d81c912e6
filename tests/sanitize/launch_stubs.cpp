// Stand-ins for the kernel launchers, so that the host code can be linked
// and exercised under the sanitizers without the device code: every launch
// reports that no device is present.
#include "kp_launch.h"

namespace kp {

hipError_t launch_prep(const ProbDev &, hipStream_t, const float *) { return hipErrorNoDevice; }
const char *stage_name(Stage) { return "stub"; }
int iteration_stages(const ProbDev &, bool, Stage[ST_COUNT]) { return 0; }
hipError_t launch_stage(const ProbDev &, hipStream_t, Stage, bool, const LaunchCfg &) { return hipErrorNoDevice; }
hipError_t launch_iteration(const ProbDev &, hipStream_t, bool, const LaunchCfg &) { return hipErrorNoDevice; }
void build_tables(Batch &, const std::vector<ProbDev> &, const LaunchCfg &) {}
int batch_stages(const std::vector<ProbDev> &, bool, Stage[ST_COUNT]) { return 0; }
hipError_t launch_stage_batch(const Batch &, hipStream_t, Stage, bool, const LaunchCfg &) { return hipErrorNoDevice; }
hipError_t launch_labels(const ProbDev &, hipStream_t, int *) { return hipErrorNoDevice; }
hipError_t launch_centroids_out(const ProbDev &, hipStream_t, float *, double *) { return hipErrorNoDevice; }
hipError_t noalloc_scratch_setup(int) { return hipErrorNoDevice; }
void *noalloc_scratch(int) { return nullptr; }
hipError_t launch_serve(const ProbDev &, hipStream_t, const LaunchCfg &, const float *, long long, int *, void *)
{
    return hipErrorNoDevice;
}
hipError_t launch_probe(const ProbDev &, hipStream_t, const float *, long long, int, float *, float *)
{
    return hipErrorNoDevice;
}
hipError_t launch_bounds(const ProbDev &, hipStream_t, const int *, long long, float *, float *, float *, int *)
{
    return hipErrorNoDevice;
}

}  // namespace kp
