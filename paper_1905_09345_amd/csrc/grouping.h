// Host-side grouping of centroids into the slot layout used by the kernels.
#pragma once
#include <cstdint>
#include <vector>

namespace kp {

constexpr int CHUNK_SLOTS = 16;   // groups are padded to a multiple of this

struct Grouping {
    int g = 0;                    // groups actually formed (min(g, k))
    int kg = 0;                   // slots including padding
    int maxgs = 0;                // largest group
    std::vector<int> perm;        // slot -> original index or -1
    std::vector<int> slot_group;  // slot -> group or -1
    std::vector<int> gstart;      // g + 1 slot offsets
    std::vector<int> gsize;       // members per group
};

// Group the k centroids (k x d FP32, row-major) into g groups; with
// chunk_medoids the first slot of every 16-slot chunk holds the chunk's
// medoid, otherwise slots ascend by original index within a group.
Grouping make_groups(const float *C, int k, int d, int g, uint64_t seed, bool chunk_medoids);

}  // namespace kp
