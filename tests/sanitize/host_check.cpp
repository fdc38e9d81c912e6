// Host code of the library under AddressSanitizer and
// UndefinedBehaviorSanitizer: argument validation and workspace planning of
// the C ABI (kp_workspace_bytes, kp_strerror, kp_last_error, kp_destroy on
// NULL) and the grouping of the initial centroids, checked against its
// invariants on random and degenerate inputs.  Nothing here touches a GPU:
// the kernel launchers are replaced by stubs at link time.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <random>
#include <vector>

#include "grouping.h"
#include "kp.h"

static int g_fails = 0;
#define CHECK(c)                                                                 \
    do {                                                                         \
        if (!(c)) {                                                              \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++g_fails;                                                           \
        }                                                                        \
    } while (0)

static kp_problem prob(int64_t n, int d, int k, int g, int prec)
{
    kp_problem p;
    std::memset(&p, 0, sizeof p);
    p.n = n;
    p.d = d;
    p.k = k;
    p.g = g;
    p.precision = prec;
    p.seed = 7;
    // planning checks the device pointers (non-NULL, 16-byte aligned) but
    // never dereferences them
    p.points_dev = reinterpret_cast<const float *>(uintptr_t{0x10000});
    p.init_centroids_dev = reinterpret_cast<const float *>(uintptr_t{0x20000});
    return p;
}

static void check_abi()
{
    for (int s = 0; s <= 6; ++s) CHECK(kp_strerror((kp_status)s) != nullptr && kp_strerror((kp_status)s)[0]);
    CHECK(kp_destroy(nullptr) == KP_OK);
    CHECK(kp_iterations(nullptr) == -1);

    CHECK(kp_workspace_bytes(nullptr, 1, nullptr) == 0);
    CHECK(std::strlen(kp_last_error()) > 0);
    kp_problem ok32 = prob(10000, 8, 16, 2, KP_PREC_FP32);
    CHECK(kp_workspace_bytes(&ok32, 0, nullptr) == 0);
    CHECK(kp_workspace_bytes(&ok32, 4097, nullptr) == 0);
    const size_t b32 = kp_workspace_bytes(&ok32, 1, nullptr);
    CHECK(b32 > 0);
    kp_problem np = ok32;
    np.points_dev = nullptr;
    CHECK(kp_workspace_bytes(&np, 1, nullptr) == 0);
    np = ok32;
    np.points_dev = reinterpret_cast<const float *>(uintptr_t{0x10004});
    CHECK(kp_workspace_bytes(&np, 1, nullptr) == 0);

    // BF16 form at the C3 and C5 shapes, every bound layout, deterministic or not
    const kp_problem shapes[2] = {prob(4000000, 128, 1024, 100, KP_PREC_BF16_RECHECK),
                                  prob(16000000, 256, 4096, 410, KP_PREC_BF16_RECHECK)};
    for (const kp_problem &p : shapes) {
        kp_tuning t;
        std::memset(&t, 0, sizeof t);
        t.bound_codes = 1;
        const size_t f32 = kp_workspace_bytes(&p, 1, &t);
        t.bound_codes = 2;
        const size_t f16 = kp_workspace_bytes(&p, 1, &t);
        t.deterministic = 1;
        const size_t det = kp_workspace_bytes(&p, 1, &t);
        CHECK(f32 > 0 && f16 > 0 && f16 < f32 && det >= f16);
        // the bound rows dominate: at least n * g * 2 bytes with codes
        CHECK(f16 >= (size_t)p.n * (size_t)p.g * 2);
    }

    // every rejected field leaves a message and no size
    const kp_problem bad[] = {prob(0, 8, 1, 1, 0),        prob(10, 0, 2, 1, 0),      prob(10, 1025, 2, 1, 0),
                              prob(10, 8, 11, 1, 0),      prob(10, 8, 4, 5, 0),      prob(10, 8, 4, 0, 0),
                              prob(1ll << 31, 8, 4, 1, 0), prob(100000, 8, 65537, 2, 0), prob(10, 8, 4, 2, 7)};
    for (const kp_problem &p : bad) {
        CHECK(kp_workspace_bytes(&p, 1, nullptr) == 0);
        CHECK(std::strlen(kp_last_error()) > 0);
    }
    struct Field {
        int32_t kp_tuning::*f;
        int32_t v;
    } badt[] = {{&kp_tuning::waves_per_block, 5},  {&kp_tuning::waves_per_block, -1}, {&kp_tuning::blocks_per_cu, 65},
                {&kp_tuning::chunk_depth, 2},      {&kp_tuning::bound_codes, 3},      {&kp_tuning::use_graph, 3},
                {&kp_tuning::timing, 2},           {&kp_tuning::timing_stages, -1},   {&kp_tuning::timing_stages, 1 << 9},
                {&kp_tuning::deterministic, 2},    {&kp_tuning::deterministic, -1},   {&kp_tuning::local_filter, 2},
                {&kp_tuning::local_filter, -1},    {&kp_tuning::plain, 2}};
    for (const Field &b : badt) {
        kp_tuning t;
        std::memset(&t, 0, sizeof t);
        t.*(b.f) = b.v;
        CHECK(kp_workspace_bytes(&ok32, 1, &t) == 0);
    }
    {
        kp_tuning t;
        std::memset(&t, 0, sizeof t);
        t.use_graph = 2;
        CHECK(kp_workspace_bytes(&ok32, 1, &t) > 0);
        t.timing = 1;   // one graph per call has no stage events
        CHECK(kp_workspace_bytes(&ok32, 1, &t) == 0);
    }

    // a batch of uneven problems needs at least the sum of its members
    std::mt19937_64 rng(3);
    std::vector<kp_problem> batch;
    size_t sum = 0;
    for (int i = 0; i < 64; ++i) {
        const int d = 8 << (rng() % 4), k = 16 << (rng() % 3);
        const int64_t n = k + (int64_t)(rng() % 200000);
        batch.push_back(prob(n, d, k, (k + 9) / 10, (int)(rng() % 2)));
        sum += kp_workspace_bytes(&batch.back(), 1, nullptr);
    }
    const size_t all = kp_workspace_bytes(batch.data(), (int32_t)batch.size(), nullptr);
    CHECK(all >= sum);
    // the largest sizes do not overflow the 64-bit sums
    const kp_problem big = prob(0x7FFFFFFFll, 1024, 65536, 65536, KP_PREC_FP32);
    const size_t bb = kp_workspace_bytes(&big, 1, nullptr);
    CHECK(bb > (size_t)0x7FFFFFFFll * 1024u);
}

static double dist(const float *a, const float *b, int d)
{
    double s = 0.0;
    for (int e = 0; e < d; ++e) {
        const double t = (double)a[e] - (double)b[e];
        s += t * t;
    }
    return std::sqrt(s);
}

static void check_grouping(const std::vector<float> &C, int k, int d, int g, uint64_t seed, bool medoids)
{
    const kp::Grouping G = kp::make_groups(C.data(), k, d, g, seed, medoids);
    const int ge = g < k ? g : k;
    CHECK(G.g == ge);
    CHECK(G.kg % kp::CHUNK_SLOTS == 0);
    CHECK((int)G.perm.size() == G.kg && (int)G.slot_group.size() == G.kg);
    CHECK((int)G.gstart.size() == G.g + 1 && (int)G.gsize.size() == G.g);
    if (g_fails) return;
    std::vector<int> seen(k, 0);
    int maxgs = 0, members = 0;
    for (int q = 0; q < G.g; ++q) {
        CHECK(G.gstart[q] % kp::CHUNK_SLOTS == 0);
        CHECK(G.gsize[q] >= 1);   // empty groups are refilled
        const int span = (G.gsize[q] + kp::CHUNK_SLOTS - 1) / kp::CHUNK_SLOTS * kp::CHUNK_SLOTS;
        CHECK(G.gstart[q + 1] == G.gstart[q] + span);
        maxgs = G.gsize[q] > maxgs ? G.gsize[q] : maxgs;
        members += G.gsize[q];
        for (int s = G.gstart[q]; s < G.gstart[q + 1]; ++s) {
            const bool real = s < G.gstart[q] + G.gsize[q];
            CHECK(real ? (G.perm[s] >= 0 && G.perm[s] < k && G.slot_group[s] == q)
                       : (G.perm[s] == -1 && G.slot_group[s] == -1));
            if (real && G.perm[s] >= 0 && G.perm[s] < k) seen[G.perm[s]]++;
        }
        // slot order within each chunk
        for (int c0 = 0; c0 < G.gsize[q]; c0 += kp::CHUNK_SLOTS) {
            const int s0 = G.gstart[q] + c0, m = std::min(kp::CHUNK_SLOTS, G.gsize[q] - c0);
            if (medoids) {
                // the first slot holds a member of least summed distance
                double best = std::numeric_limits<double>::infinity(), first = 0.0;
                for (int i = 0; i < m; ++i) {
                    double tot = 0.0;
                    for (int j = 0; j < m; ++j)
                        tot += dist(&C[(size_t)G.perm[s0 + i] * d], &C[(size_t)G.perm[s0 + j] * d], d);
                    if (i == 0) first = tot;
                    best = tot < best ? tot : best;
                }
                CHECK(first <= best * (1.0 + 1e-12));
            } else {
                for (int i = 1; i < m; ++i) CHECK(G.perm[s0 + i - 1] < G.perm[s0 + i]);
            }
        }
    }
    CHECK(G.gstart[G.g] == G.kg);
    CHECK(G.maxgs == maxgs && members == k);
    for (int j = 0; j < k; ++j) CHECK(seen[j] == 1);
    // sizes capped at the smallest chunk multiple holding k / g
    const int cap = kp::CHUNK_SLOTS * ((k + ge * kp::CHUNK_SLOTS - 1) / (ge * kp::CHUNK_SLOTS));
    if (ge < k) CHECK(maxgs <= cap);
}

static void check_groupings()
{
    std::mt19937_64 rng(11);
    std::normal_distribution<float> nd(0.f, 1.f);
    const int ks[] = {1, 2, 5, 16, 17, 100, 1000};
    const int ds[] = {1, 3, 8, 64};
    for (int k : ks)
        for (int d : ds) {
            std::vector<float> C((size_t)k * d);
            for (float &v : C) v = nd(rng) * 10.f;
            const int gs[] = {1, 2, (k + 9) / 10, k};
            for (int g : gs)
                for (int med = 0; med < 2; ++med) check_grouping(C, k, d, g, rng(), med != 0);
        }
    // degenerate: identical centroids, and two far clusters of unequal size
    std::vector<float> same((size_t)300 * 4, 1.5f);
    check_grouping(same, 300, 4, 30, 1, true);
    check_grouping(same, 300, 4, 30, 1, false);
    std::vector<float> two((size_t)200 * 2);
    for (int j = 0; j < 200; ++j) {
        two[2 * j] = (j < 190 ? 0.f : 1e6f) + nd(rng);
        two[2 * j + 1] = nd(rng);
    }
    check_grouping(two, 200, 2, 20, 5, true);
}

int main()
{
    check_abi();
    check_groupings();
    if (g_fails) {
        std::fprintf(stderr, "%d checks failed\n", g_fails);
        return 1;
    }
    std::printf("host checks passed\n");
    return 0;
}
