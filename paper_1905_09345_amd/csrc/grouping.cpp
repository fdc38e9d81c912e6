// Grouping of the initial centroids (host, once per kp_init).
//
// The group-level filter keeps one lower bound per (point, group of
// centroids) (paper, Section 1: "Group-level Filter").  The paper does not
// say how groups are formed; here they are the clusters of a small FP64
// K-means over the k initial centroids: k-means++ seeding from the problem's
// seed, five Lloyd iterations, every empty group filled with the member of
// the largest group that lies farthest from that group's center, and group
// sizes capped at the smallest multiple of 16 (one matrix-core chunk) that
// holds k / g, and (BF16 problems) the medoid of every chunk in its first
// slot.  The grouping only changes how much work the filter saves and how
// tight the BF16 error bounds are, never the result.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <limits>
#include <vector>

#include "grouping.h"

namespace kp {

namespace {

struct SplitMix {
    uint64_t s;
    uint64_t next()
    {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return (double)(next() >> 11) * 0x1.0p-53; }
};

double sq(const float *a, const double *b, int d)
{
    double s = 0.0;
    for (int i = 0; i < d; ++i) {
        double t = (double)a[i] - b[i];
        s += t * t;
    }
    return s;
}

}  // namespace

Grouping make_groups(const float *C, int k, int d, int g, uint64_t seed, bool chunk_medoids)
{
    std::vector<int> lab(k, 0);
    if (g >= k) {
        for (int j = 0; j < k; ++j) lab[j] = j;
        g = k;
    } else if (g > 1) {
        SplitMix rng{seed ^ 0x6B70796E71ull};
        std::vector<double> ctr((size_t)g * d);
        std::vector<double> best(k, std::numeric_limits<double>::infinity());
        int first = (int)(rng.next() % (uint64_t)k);
        for (int i = 0; i < d; ++i) ctr[i] = C[(size_t)first * d + i];
        for (int q = 1; q < g; ++q) {
            double tot = 0.0;
            for (int j = 0; j < k; ++j) {
                best[j] = std::min(best[j], sq(C + (size_t)j * d, &ctr[(size_t)(q - 1) * d], d));
                tot += best[j];
            }
            int pick = (int)(rng.next() % (uint64_t)k);
            if (tot > 0.0) {
                double u = rng.uniform() * tot, acc = 0.0;
                for (int j = 0; j < k; ++j) {
                    acc += best[j];
                    if (acc > u) {
                        pick = j;
                        break;
                    }
                }
            }
            for (int i = 0; i < d; ++i) ctr[(size_t)q * d + i] = C[(size_t)pick * d + i];
        }
        std::vector<int> cnt(g);
        for (int it = 0; it < 5; ++it) {
            for (int j = 0; j < k; ++j) {
                double bv = std::numeric_limits<double>::infinity();
                int bq = 0;
                for (int q = 0; q < g; ++q) {
                    double v = sq(C + (size_t)j * d, &ctr[(size_t)q * d], d);
                    if (v < bv) {
                        bv = v;
                        bq = q;
                    }
                }
                lab[j] = bq;
            }
            std::fill(ctr.begin(), ctr.end(), 0.0);
            std::fill(cnt.begin(), cnt.end(), 0);
            for (int j = 0; j < k; ++j) {
                cnt[lab[j]]++;
                for (int i = 0; i < d; ++i) ctr[(size_t)lab[j] * d + i] += C[(size_t)j * d + i];
            }
            for (int q = 0; q < g; ++q)
                if (cnt[q])
                    for (int i = 0; i < d; ++i) ctr[(size_t)q * d + i] /= cnt[q];
        }
        // fill empty groups
        for (;;) {
            int empty = -1, big = 0;
            for (int q = 0; q < g; ++q) {
                if (cnt[q] == 0 && empty < 0) empty = q;
                if (cnt[q] > cnt[big]) big = q;
            }
            if (empty < 0) break;
            int far = -1;
            double fv = -1.0;
            for (int j = 0; j < k; ++j) {
                if (lab[j] != big) continue;
                double v = sq(C + (size_t)j * d, &ctr[(size_t)big * d], d);
                if (v > fv) {
                    fv = v;
                    far = j;
                }
            }
            lab[far] = empty;
            cnt[big]--;
            cnt[empty] = 1;
            for (int i = 0; i < d; ++i) ctr[(size_t)empty * d + i] = C[(size_t)far * d + i];
        }
        // cap the group sizes at the smallest multiple of the chunk that holds
        // k / g members: a group above it gives up its members farthest from
        // its center, each to the group with room whose center is nearest.
        // Every group then fills its chunks, and no visit pays for a chunk
        // holding one or two centroids.
        const int cap = CHUNK_SLOTS * ((k + g * CHUNK_SLOTS - 1) / (g * CHUNK_SLOTS));
        for (int q = 0; q < g; ++q) {
            if (cnt[q] <= cap) continue;
            std::vector<std::pair<double, int>> mem;
            for (int j = 0; j < k; ++j)
                if (lab[j] == q) mem.push_back({sq(C + (size_t)j * d, &ctr[(size_t)q * d], d), j});
            std::sort(mem.begin(), mem.end(), [](const std::pair<double, int> &x, const std::pair<double, int> &y) {
                return x.first > y.first || (x.first == y.first && x.second < y.second);
            });
            for (size_t e = 0; e < mem.size() && cnt[q] > cap; ++e) {
                const int j = mem[e].second;
                int to = -1;
                double tv = std::numeric_limits<double>::infinity();
                for (int r = 0; r < g; ++r) {
                    if (r == q || cnt[r] >= cap) continue;
                    const double v = sq(C + (size_t)j * d, &ctr[(size_t)r * d], d);
                    if (v < tv) {
                        tv = v;
                        to = r;
                    }
                }
                if (to < 0) break;   // unreachable: g * cap >= k
                lab[j] = to;
                cnt[q]--;
                cnt[to]++;
            }
        }
    }
    Grouping out;
    out.g = g;
    out.gsize.assign(g, 0);
    for (int j = 0; j < k; ++j) out.gsize[lab[j]]++;
    out.gstart.assign(g + 1, 0);
    int run = 0;
    out.maxgs = 0;
    for (int q = 0; q < g; ++q) {
        out.gstart[q] = run;
        run += (out.gsize[q] + CHUNK_SLOTS - 1) / CHUNK_SLOTS * CHUNK_SLOTS;
        out.maxgs = std::max(out.maxgs, out.gsize[q]);
    }
    out.gstart[g] = run;
    out.kg = run;
    out.perm.assign(run, -1);
    out.slot_group.assign(run, -1);
    std::vector<int> fill(g, 0);
    for (int j = 0; j < k; ++j) {   // ascending original index within a group
        int q = lab[j];
        int s = out.gstart[q] + fill[q]++;
        out.perm[s] = j;
        out.slot_group[s] = q;
    }
    // The first slot of every chunk is the reference the kernels express the
    // chunk's other rows against (their products and error bounds scale with
    // the distance to it): move the chunk's medoid there, the member with the
    // least summed distance to the others (the lowest original index among
    // equals).  A far member then costs precision in its own row only.
    for (int q = 0; chunk_medoids && q < g; ++q) {
        for (int c0 = 0; c0 < out.gsize[q]; c0 += CHUNK_SLOTS) {
            const int s0 = out.gstart[q] + c0, m = std::min(CHUNK_SLOTS, out.gsize[q] - c0);
            int best = 0;
            double bv = std::numeric_limits<double>::infinity();
            for (int i = 0; i < m; ++i) {
                const float *ci = C + (size_t)out.perm[s0 + i] * d;
                double tot = 0.0;
                for (int j = 0; j < m; ++j) {
                    if (j == i) continue;
                    const float *cj = C + (size_t)out.perm[s0 + j] * d;
                    double t2 = 0.0;
                    for (int e = 0; e < d; ++e) {
                        const double t = (double)ci[e] - (double)cj[e];
                        t2 += t * t;
                    }
                    tot += std::sqrt(t2);
                }
                if (tot < bv) {   // members ascend by original index, so the first of equals stays
                    bv = tot;
                    best = i;
                }
            }
            std::swap(out.perm[s0], out.perm[s0 + best]);
        }
    }
    return out;
}

}  // namespace kp
