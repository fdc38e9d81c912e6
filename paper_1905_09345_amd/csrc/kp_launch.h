// Host-side launchers of the kernels in kp_kernels.hip (internal to libkp).
#pragma once
#include <hip/hip_runtime.h>
#include <vector>
#include "kp_device.h"

namespace kp {

struct LaunchCfg {
    int waves;      // waves of 64 lanes per workgroup of the assignment kernels
    int grid_cap;   // upper bound on workgroups of grid-stride kernels
    int depth;      // centroid chunks in flight per workgroup (BF16 mode): 1 or 3
    bool lb16;      // BF16 mode: group bounds stored as FP16 codes
};

// Per-point BF16 shadow and norms, initial centroid rows, drift rings at t=0.
hipError_t launch_prep(const ProbDev &P, hipStream_t s, const float *init_dev);
// Stages of one iteration, in launch order.
enum Stage {
    ST_BEGIN = 0, ST_FILTER, ST_SORT, ST_ASSIGN_DENSE, ST_GFILTER, ST_ASSIGN, ST_RECHECK, ST_UPDATE, ST_CENTROIDS,
    ST_COUNT
};
const char *stage_name(Stage st);
// The stages of a dense (first) or filtered iteration of problem P, in order.
int iteration_stages(const ProbDev &P, bool dense, Stage out[ST_COUNT]);
// Launch the kernels of one stage.
hipError_t launch_stage(const ProbDev &P, hipStream_t s, Stage st, bool dense, const LaunchCfg &cfg);
// One K-means iteration (dense = every distance) of one problem.
hipError_t launch_iteration(const ProbDev &P, hipStream_t s, bool dense, const LaunchCfg &cfg);
// ---------------------------------------------------------------- batches
// A ctx with several problems launches each stage once for all of them.
// Table id (a launch shape, per template class where the kernel has one)
// gives each problem a contiguous range of blocks; a problem outside the
// class gets none.
enum TabId {
    TB_BEGIN = 0, TB_FILTER, TB_SORT, TB_ONE, TB_CENT, TB_GT, TB_GF, TB_HIST, TB_SCATTER, TB_ATAB, TB_ROWPRE,
    TB_DENSE_F32,                     // + DMAX class (5)
    TB_TILE_F32 = TB_DENSE_F32 + 5,   // + DMAX class (5)
    TB_BLK64 = TB_TILE_F32 + 5,       // + KS class (6)
    TB_RECHECK = TB_BLK64 + 6,        // + NV class (4)
    TB_SEGSUM = TB_RECHECK + 4,       // + DCH class (6)
    TB_COUNT = TB_SEGSUM + 6
};
struct Batch {
    int count = 0;
    const ProbDev *probs = nullptr;   // device copy of the problems
    const int *tabs = nullptr;        // device: TB_COUNT tables of count + 1 block offsets
    std::vector<int> htabs;           // host copy
    int total(int id) const { return htabs[(size_t)id * (count + 1) + count]; }
    const int *tab(int id) const { return tabs + (size_t)id * (count + 1); }
};
// Block offsets of every table for these problems (host side).
void build_tables(Batch &B, const std::vector<ProbDev> &hp, const LaunchCfg &cfg);
// The stages of one iteration of a batch, in order.
int batch_stages(const std::vector<ProbDev> &hp, bool dense, Stage out[ST_COUNT]);
// Launch one stage for every problem of the batch.
hipError_t launch_stage_batch(const Batch &B, hipStream_t s, Stage st, bool dense, const LaunchCfg &cfg);

// Current assignment as original centroid indices.
hipError_t launch_labels(const ProbDev &P, hipStream_t s, int *out);
// Current centroids in original order (either output may be null).
hipError_t launch_centroids_out(const ProbDev &P, hipStream_t s, float *c32, double *c64);
// Serving: labels of nq query rows against the problem's current centroids.
// Largest slot count that keeps anchor tables (the per-anchor squared
// distances Qt: kg^2 FP32 <= 1 GiB), and with them the anchored estimates of
// the filtered iterations and of serving's second pass.
constexpr size_t ANCHOR_MAX_SLOTS = 16384;
// scratch: a SERVE_HEADER-byte header (the BF16 passes' uncertain-query
// counters and nq), the list of uncertain queries (4 nq bytes); with anchors
// also the anchors or provisional slots (4 nq), the list sorted by slot (8 nq) and a
// slot histogram and its scan (2 x 4 (ANCHOR_MAX_SLOTS + 1)), each rounded up
// to 256 bytes.
constexpr size_t SERVE_HEADER = 256;
constexpr size_t serve_up(size_t v) { return (v + 255) / 256 * 256; }
constexpr size_t serve_scratch_bytes(long long nq, bool anchored)
{
    return SERVE_HEADER + serve_up((size_t)nq * 4) +
           (anchored ? serve_up((size_t)nq * 4) + serve_up((size_t)nq * 8) + serve_up(8 * (ANCHOR_MAX_SLOTS + 1)) : 0);
}
// Serving without allocation: the largest query count of kp_predict_noalloc,
// whose scratch is a fixed per-device array inside the library.
constexpr long long NOALLOC_MAX_QUERIES = 1ll << 22;
// Once per device, with that device current: take the device address of the
// fixed scratch array and keep it.  The address for a device after setup
// (nullptr before).
hipError_t noalloc_scratch_setup(int device);
void *noalloc_scratch(int device);
hipError_t launch_serve(const ProbDev &P, hipStream_t s, const LaunchCfg &cfg, const float *Q, long long nq,
                        int *labels, void *scratch);

// Diagnostics: BF16x3 estimates and bounds of query rows against every
// centroid (est, eta: nq x k, original order); bounds of listed points.
hipError_t launch_probe(const ProbDev &P, hipStream_t s, const float *Q, long long nq, int anchor, float *est,
                        float *eta);
hipError_t launch_bounds(const ProbDev &P, hipStream_t s, const int *idx, long long np, float *ub, float *lbp,
                         float *lb, int *groups);

}  // namespace kp
