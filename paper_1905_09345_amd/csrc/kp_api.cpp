// C ABI of libkp (declared in include/kp.h): argument checks, workspace
// planning, the one-time grouping of centroids, and the ordering of the
// per-iteration kernels on a stream (optionally replayed from a hipGraph).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/kp.h"
#include "grouping.h"
#include "kp_device.h"
#include "kp_launch.h"

namespace {

thread_local std::string g_last_error;

void set_error(const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

constexpr size_t ALIGN = 256;
using kp::ANCHOR_MAX_SLOTS;
inline size_t up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Byte offsets of one problem's arrays inside the workspace.
struct Plan {
    size_t xn, st, lb, c32, cb, cbl, cn, c64, sums, delta, cnt, perm, sgrp, gstart, gsize;
    size_t Sc, Sg, Sd, Scu, Scd, Sgu, Sgd, slk, nrel, Wu, Qt, Wa, Sdud, L1, L1s, L1x, L3, minnc, tlist, tcnt, ps4, psf, mvp, mvo, mvn, srtp, srtk, hist, cursor, hist1,
        cursor1, ctr, rowt, rclosed, stats, iter, sink, lbsc, dcnt, doff, hist2, spart, pfirst, plast;
    size_t bytes;
    int kgmax, ldc, ldb, gs;
    bool anch;       // BF16 filtered tiles use estimates relative to an anchor centroid
    size_t nk1max;   // keys of the L1 order for kgmax slots
};

Plan plan_problem(const kp_problem &p, bool lb16, bool det)
{
    Plan o;
    const size_t n = (size_t)p.n;
    const int d = p.d, g = p.g;
    const bool bf = p.precision == KP_PREC_BF16_RECHECK;
    o.kgmax = p.k + (kp::CHUNK_SLOTS - 1) * g;
    // L1 ordered by slot, then by a bucket of the nearest other group: at most
    // max(slots, L1_HIST) keys whatever the final slot count
    o.nk1max = (size_t)(o.kgmax > kp::L1_HIST ? o.kgmax : kp::L1_HIST);
    o.ldc = (d + 3) / 4 * 4;
    o.ldb = (d + 31) / 32 * 32;
    if (o.ldb == 160) o.ldb = 192;   // BF16 tiles take 1, 2, 3, 4, 6 or 8 steps of 32
    if (o.ldb == 224) o.ldb = 256;
    // bound row stride: FP32 mode 16-byte rows; BF16 mode 128-byte rows (one
    // cache line per 64 FP16 codes or 32 FP32 bounds, so that a row's reads
    // touch no line it does not need)
    o.gs = bf ? (lb16 ? (g + 63) / 64 * 64 : (g + 31) / 32 * 32) : (g + 3) / 4 * 4;
    const size_t kgm = (size_t)o.kgmax;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t r = off;
        off += up(bytes ? bytes : 1, ALIGN);
        return r;
    };
    o.xn = take(bf ? n * 4 : 0);
    o.st = take(n * sizeof(kp::PointState));
    o.lb = take(n * (size_t)o.gs * (bf && lb16 ? 2 : 4));   // FP16 codes or FP32
    o.c32 = take(kgm * o.ldc * 4);
    o.cb = take(bf ? kgm * o.ldb * 2 : 0);
    o.cbl = take(bf ? kgm * o.ldb * 2 : 0);
    o.cn = take(kgm * 4);
    o.c64 = take(kgm * d * 8);
    o.sums = take(kgm * d * 8);
    o.delta = take(kgm * 8);
    o.cnt = take(kgm * 4);
    o.perm = take(kgm * 4);
    o.sgrp = take(kgm * 4);
    o.gstart = take((size_t)(g + 1) * 4);
    o.gsize = take((size_t)g * 4);
    o.Sc = take(kgm * 8);
    o.Sg = take((size_t)g * 8);
    o.Sd = take(8);
    o.Scu = take(kgm * 4);
    o.Scd = take(kgm * 4);
    o.Sgu = take((size_t)g * 4);
    o.Sgd = take((size_t)g * 4);
    o.slk = take(kgm * 4);
    // BF16 mode: relative norms and per-chunk bounds of the chunk rows; with
    // anchors, the slot-to-slot table of squared distances and the
    // per-(anchor, chunk) bounds (kgmax <= ANCHOR_MAX_SLOTS keeps them <= 1 GiB)
    const size_t nchm = kgm / kp::CHUNK;
    o.anch = bf && kgm <= ANCHOR_MAX_SLOTS;
    o.nrel = take(bf ? kgm * 4 : 0);
    o.Wu = take(bf ? nchm * 8 : 0);
    o.Qt = take(o.anch ? kgm * kgm * 4 : 0);
    o.Wa = take(o.anch ? kgm * nchm * 8 : 0);
    o.Sdud = take(8);
    o.L1 = take(n * 16);
    o.L1s = take(n * 4);
    o.L1x = take(bf ? n * 16 : 0);
    o.L3 = take(bf ? n * 4 : 0);
    o.minnc = take(bf ? n * 4 : 0);
    const size_t ntiles = (n + 63) / 64;
    o.tlist = take(ntiles * (size_t)g * 16);   // per-tile visit lists of the group filter
    o.tcnt = take(ntiles * 4);
    o.ps4 = take(n * 16);
    o.psf = take(n * 4);
    o.mvp = take(n * 4);
    o.mvo = take(n * 4);
    o.mvn = take(n * 4);
    o.srtp = take(2 * n * 4);
    o.srtk = take(2 * n * 4);
    o.hist = take((kgm + 1) * 4);
    o.cursor = take((kgm + 1) * 4);
    o.hist1 = take((o.nk1max + 1) * 4);
    o.cursor1 = take((o.nk1max + 1) * 4);
    o.ctr = take(kp::NCTR * 8);
    o.rowt = take(4);
    o.rclosed = take((n + 63) / 64 * 8);
    o.stats = take((size_t)kp::STATS_CAP * 16 * 8);
    o.iter = take(4);
    o.sink = take(bf ? (size_t)kp::SINK_SLOTS * 64 : 0);
    o.lbsc = take(16);
    // deterministic mode: per-chunk failure counts and offsets, the (key,
    // block) table of the stable sorts, the scan's partial sums and the
    // pieces' partial centroid sums
    const size_t nchunks = (n + kp::BF_CHUNK - 1) / kp::BF_CHUNK;
    const size_t nkeys = std::max(o.nk1max, kgm);
    const size_t npieces = (n + kp::DS_PIECE - 1) / kp::DS_PIECE;
    o.dcnt = take(det ? nchunks * 4 : 0);
    o.doff = take(det ? nchunks * 4 : 0);
    o.hist2 = take(det ? nkeys * kp::SS_NB * 4 : 0);
    o.spart = take(det ? (size_t)kp::SS_SCAN_BLOCKS * 4 : 0);
    o.pfirst = take(det ? npieces * d * 8 : 0);
    o.plast = take(det ? npieces * d * 8 : 0);
    o.bytes = off;
    return o;
}

// Bits needed for keys 0..maxkey.
int bits_for(int maxkey)
{
    int b = 0;
    while (b < 31 && (1 << b) <= maxkey) ++b;
    return b;
}

bool validate(const kp_problem *ps, int32_t count, const kp_tuning *t)
{
    if (!ps) {
        set_error("problems is NULL");
        return false;
    }
    if (count < 1 || count > 4096) {
        set_error("count=%d outside 1..4096", count);
        return false;
    }
    if (t) {
        if (t->waves_per_block < 0 || t->waves_per_block > 4) {
            set_error("waves_per_block=%d outside 0..4", t->waves_per_block);
            return false;
        }
        if (t->blocks_per_cu < 0 || t->blocks_per_cu > 64) {
            set_error("blocks_per_cu=%d outside 0..64", t->blocks_per_cu);
            return false;
        }
        if (t->chunk_depth != 0 && t->chunk_depth != 1 && t->chunk_depth != 3) {
            set_error("chunk_depth=%d not 0, 1 or 3", t->chunk_depth);
            return false;
        }
        if (t->bound_codes < 0 || t->bound_codes > 2) {
            set_error("bound_codes=%d outside 0..2", t->bound_codes);
            return false;
        }
        if (t->use_graph < -1 || t->use_graph > 2) {
            set_error("use_graph=%d outside -1..2", t->use_graph);
            return false;
        }
        if (t->use_graph == 2 && t->timing) {
            set_error("use_graph=2 (one graph per kp_iterate call) records no stage events; set timing=0");
            return false;
        }
        if (t->timing_stages < 0 || t->timing_stages >= (1 << kp::ST_COUNT)) {
            set_error("timing_stages=%d outside 0..%d", t->timing_stages, (1 << kp::ST_COUNT) - 1);
            return false;
        }
        if (t->timing < 0 || t->timing > 1) {
            set_error("timing=%d outside 0..1", t->timing);
            return false;
        }
        if (t->deterministic < 0 || t->deterministic > 1) {
            set_error("deterministic=%d outside 0..1", t->deterministic);
            return false;
        }
        if (t->local_filter < 0 || t->local_filter > 1) {
            set_error("local_filter=%d outside 0..1", t->local_filter);
            return false;
        }
        if (t->plain < 0 || t->plain > 1) {
            set_error("plain=%d outside 0..1", t->plain);
            return false;
        }
    }
    for (int i = 0; i < count; ++i) {
        const kp_problem &p = ps[i];
        if (p.n < 1 || p.n > 0x7FFFFFFFll) {
            set_error("problem %d: n=%lld outside 1..2^31-1", i, (long long)p.n);
            return false;
        }
        if (p.d < 1 || p.d > 1024) {
            set_error("problem %d: d=%d outside 1..1024", i, p.d);
            return false;
        }
        if (p.k < 1 || p.k > 65536 || (int64_t)p.k > p.n) {
            set_error("problem %d: k=%d must satisfy 1 <= k <= min(n, 65536)", i, p.k);
            return false;
        }
        if (p.g < 1 || p.g > p.k) {
            set_error("problem %d: g=%d must satisfy 1 <= g <= k", i, p.g);
            return false;
        }
        if (p.precision != KP_PREC_FP32 && p.precision != KP_PREC_BF16_RECHECK) {
            set_error("problem %d: unknown precision %d", i, p.precision);
            return false;
        }
        if (!p.points_dev || !p.init_centroids_dev) {
            set_error("problem %d: NULL points or initial centroids", i);
            return false;
        }
        if (((uintptr_t)p.points_dev & 15u) != 0) {
            set_error("problem %d: points_dev must be 16-byte aligned", i);
            return false;
        }
    }
    return true;
}

bool supported(const kp_problem *ps, int32_t count)
{
    for (int i = 0; i < count; ++i) {
        const kp_problem &p = ps[i];
        if (p.precision == KP_PREC_FP32 && p.d > 128) {
            set_error("problem %d: FP32 mode supports d <= 128 (got %d); use BF16_RECHECK", i, p.d);
            return false;
        }
        if (p.precision == KP_PREC_BF16_RECHECK && p.d > 256) {
            set_error("problem %d: BF16 mode supports d <= 256 (got %d)", i, p.d);
            return false;
        }
        if (p.precision == KP_PREC_BF16_RECHECK && p.g > 1024) {
            set_error("problem %d: BF16 mode supports g <= 1024 (got %d)", i, p.g);
            return false;
        }
    }
    return true;
}

}  // namespace

struct kp_ctx;
static void release_ctx(kp_ctx *ctx);

// HIP event pairs recorded around stage launches on the ctx's own stream.
struct StageTimer {
    static constexpr int NSTAGE = kp::ST_COUNT + 1;   // + one entry per graph replay
    struct Rec {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
    std::vector<Rec> pending;
    double ms[NSTAGE] = {};
    long long launches[NSTAGE] = {};
    static const char *name(int st) { return st == kp::ST_COUNT ? "filtered_iter" : kp::stage_name((kp::Stage)st); }
    hipError_t begin(int stage, hipStream_t s, Rec &r)
    {
        r.stage = stage;
        if (pool.empty()) {
            hipEvent_t a, b;
            hipError_t e = hipEventCreate(&a);
            if (e != hipSuccess) return e;
            e = hipEventCreate(&b);
            if (e != hipSuccess) {
                (void)hipEventDestroy(a);
                return e;
            }
            pool.push_back({a, b});
        }
        r.a = pool.back().first;
        r.b = pool.back().second;
        pool.pop_back();
        return hipEventRecord(r.a, s);
    }
    // a fresh event pair for a stage recorded inside a graph replay
    hipError_t take(int stage, Rec &r)
    {
        r.stage = stage;
        if (pool.empty()) {
            hipEvent_t a, b;
            hipError_t e = hipEventCreate(&a);
            if (e != hipSuccess) return e;
            e = hipEventCreate(&b);
            if (e != hipSuccess) {
                (void)hipEventDestroy(a);
                return e;
            }
            pool.push_back({a, b});
        }
        r.a = pool.back().first;
        r.b = pool.back().second;
        pool.pop_back();
        return hipSuccess;
    }
    hipError_t end(hipStream_t s, Rec &r)
    {
        hipError_t e = hipEventRecord(r.b, s);
        pending.push_back(r);
        return e;
    }
    hipError_t harvest()
    {
        for (auto &r : pending) {
            hipError_t e = hipEventSynchronize(r.b);
            if (e != hipSuccess) return e;
            float t = 0.f;
            e = hipEventElapsedTime(&t, r.a, r.b);
            if (e != hipSuccess) return e;
            ms[r.stage] += t;
            launches[r.stage] += 1;
            pool.push_back({r.a, r.b});
        }
        pending.clear();
        return hipSuccess;
    }
    void destroy()
    {
        for (auto &r : pending) pool.push_back({r.a, r.b});
        pending.clear();
        for (auto &p : pool) {
            (void)hipEventDestroy(p.first);
            (void)hipEventDestroy(p.second);
        }
        pool.clear();
    }
};

struct kp_ctx {
    int count = 0;
    int timing = 0;
    unsigned timed_stages = ~0u;   // bit s: stage s is bracketed by events when timing is on
    StageTimer timer;
    int device = 0;
    hipStream_t user = nullptr, own = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::vector<kp::ProbDev> P;
    std::vector<std::vector<int>> slot_of;    // per problem: original centroid index -> slot
    kp::Batch batch;                           // count > 1: batched launches
    kp::LaunchCfg cfg{4, 4096, 1, false};
    int use_graph = 1;
    int plain = 0;   // plain Lloyd: a dense pass in every iteration
    int iters = 0;
    bool poisoned = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    // use_graph = 2: every iteration of a kp_iterate call in one graph, kept
    // for the next call of the same shape (iteration count, dense first)
    hipGraphExec_t rexec = nullptr;
    int run_iters = 0;
    bool run_dense = false;
    // timing inside the graph: event-record nodes around each stage, pointed
    // at fresh events before every replay
    std::vector<hipEvent_t> cap_events;        // placeholders recorded at capture
    std::vector<hipGraphNode_t> ev_nodes;      // 2 per timed stage: begin, end
    std::vector<int> ev_stage;
};

// Frees the ctx's host resources, stream, events and graph without touching
// the caller-visible error string.
static void release_ctx(kp_ctx *ctx)
{
    if (!ctx) return;
    if (ctx->own) (void)hipStreamSynchronize(ctx->own);
    ctx->timer.destroy();
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    if (ctx->rexec) (void)hipGraphExecDestroy(ctx->rexec);
    for (hipEvent_t e : ctx->cap_events) (void)hipEventDestroy(e);
    if (ctx->ev_in) (void)hipEventDestroy(ctx->ev_in);
    if (ctx->ev_out) (void)hipEventDestroy(ctx->ev_out);
    if (ctx->own) (void)hipStreamDestroy(ctx->own);
    delete ctx;
}

#define KP_HIP(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            set_error("%s failed: %s", #expr, hipGetErrorString(e_));                  \
            if (ctx) ctx->poisoned = true;                                             \
            return KP_ERR_HIP;                                                         \
        }                                                                              \
    } while (0)

extern "C" {

static size_t batch_header_bytes(int count);

size_t kp_workspace_bytes(const kp_problem *problems, int32_t count, const kp_tuning *tuning)
{
    if (!validate(problems, count, tuning)) return 0;
    size_t total = 0;
    const bool lb16 = tuning && tuning->bound_codes == 2;
    const bool det = tuning && tuning->deterministic == 1;
    for (int i = 0; i < count; ++i) total += plan_problem(problems[i], lb16, det).bytes;
    return total + batch_header_bytes(count);
}

// A ctx with several problems keeps, after the problems' regions, a device
// copy of every problem descriptor and the block tables of the batched
// launches.
static size_t batch_header_bytes(int count)
{
    if (count <= 1) return 0;
    return up((size_t)count * sizeof(kp::ProbDev), ALIGN) + up((size_t)kp::TB_COUNT * (count + 1) * 4, ALIGN);
}

kp_status kp_init(kp_ctx **out, const kp_problem *problems, int32_t count, void *workspace, size_t ws_bytes,
                  void *stream, const kp_tuning *tuning)
{
    kp_ctx *ctx = nullptr;
    if (!out) {
        set_error("out is NULL");
        return KP_ERR_INVALID;
    }
    if (!validate(problems, count, tuning)) return KP_ERR_INVALID;
    if (!supported(problems, count)) return KP_ERR_UNSUPPORTED;
    if (!workspace || ((uintptr_t)workspace % ALIGN) != 0) {
        set_error("workspace must be non-NULL and %zu-byte aligned", ALIGN);
        return KP_ERR_INVALID;
    }
    std::vector<Plan> plans;
    size_t need = 0;
    const bool lb16 = tuning && tuning->bound_codes == 2;
    const bool det = tuning && tuning->deterministic == 1;
    if (det && count > 1) {
        set_error("deterministic mode runs one problem per ctx (got %d)", count);
        return KP_ERR_UNSUPPORTED;
    }
    for (int i = 0; i < count; ++i) {
        plans.push_back(plan_problem(problems[i], lb16, det));
        need += plans.back().bytes;
    }
    const size_t problem_bytes = need;
    need += batch_header_bytes(count);
    if (ws_bytes < need) {
        set_error("workspace has %zu bytes, needs %zu", ws_bytes, need);
        return KP_ERR_INVALID;
    }
    ctx = new (std::nothrow) kp_ctx;
    if (!ctx) {
        set_error("host allocation failed");
        return KP_ERR_NOMEM;
    }
    std::unique_ptr<kp_ctx, void (*)(kp_ctx *)> guard(ctx, release_ctx);   // freed on any early return
    ctx->count = count;
    ctx->user = (hipStream_t)stream;
    if (tuning) {
        if (tuning->waves_per_block) ctx->cfg.waves = tuning->waves_per_block;
        if (tuning->blocks_per_cu) ctx->cfg.grid_cap = 256 * tuning->blocks_per_cu;
        if (tuning->chunk_depth) ctx->cfg.depth = tuning->chunk_depth;
        ctx->cfg.lb16 = tuning->bound_codes == 2;
        if (tuning->use_graph) ctx->use_graph = tuning->use_graph > 0 ? tuning->use_graph : 0;
        ctx->timing = tuning->timing;
        ctx->plain = tuning->plain;
        if (tuning->timing_stages) ctx->timed_stages = (unsigned)tuning->timing_stages;
    }
    KP_HIP(hipGetDevice(&ctx->device));
    KP_HIP(kp::noalloc_scratch_setup(ctx->device));   // kp_predict_noalloc's scratch on this device
    KP_HIP(hipStreamCreateWithFlags(&ctx->own, hipStreamNonBlocking));
    KP_HIP(hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming));
    KP_HIP(hipEventCreateWithFlags(&ctx->ev_out, hipEventDisableTiming));
    KP_HIP(hipMemsetAsync(workspace, 0, need, ctx->user));

    char *base = (char *)workspace;
    std::vector<float> hc;
    for (int i = 0; i < count; ++i) {
        const kp_problem &p = problems[i];
        const Plan &o = plans[i];
        hc.resize((size_t)p.k * p.d);
        KP_HIP(hipMemcpyAsync(hc.data(), p.init_centroids_dev, hc.size() * 4, hipMemcpyDeviceToHost, ctx->user));
        KP_HIP(hipStreamSynchronize(ctx->user));
        kp::Grouping G = kp::make_groups(hc.data(), p.k, p.d, p.g, p.seed, p.precision == KP_PREC_BF16_RECHECK);
        kp::ProbDev P;
        std::memset(&P, 0, sizeof P);
        P.n = p.n;
        P.d = p.d;
        P.k = p.k;
        P.g = G.g;
        P.kg = G.kg;
        P.ldc = o.ldc;
        P.ldb = o.ldb;
        P.gs = o.gs;
        P.prec = p.precision;
        P.lb16 = (p.precision == KP_PREC_BF16_RECHECK && lb16) ? 1 : 0;
        P.maxgs = G.maxgs;
        P.nk1 = G.kg * kp::l1_buckets(p.n, G.kg, G.g);
        P.X = p.points_dev;
        P.xn = (float *)(base + o.xn);
        P.st = (kp::PointState *)(base + o.st);
        P.lb = (float *)(base + o.lb);
        P.lbh = (uint16_t *)(base + o.lb);
        P.lbsc = (float *)(base + o.lbsc);
        P.c32 = (float *)(base + o.c32);
        P.cb = (uint16_t *)(base + o.cb);
        P.cbl = (uint16_t *)(base + o.cbl);
        P.cn = (float *)(base + o.cn);
        P.c64 = (double *)(base + o.c64);
        P.sums = (double *)(base + o.sums);
        P.delta = (double *)(base + o.delta);
        P.cnt = (int *)(base + o.cnt);
        P.perm = (const int *)(base + o.perm);
        P.slot_group = (const int *)(base + o.sgrp);
        P.gstart = (const int *)(base + o.gstart);
        P.gsize = (const int *)(base + o.gsize);
        P.Sc = (double *)(base + o.Sc);
        P.Sg = (double *)(base + o.Sg);
        P.Sd = (double *)(base + o.Sd);
        P.Scu = (float *)(base + o.Scu);
        P.Scd = (float *)(base + o.Scd);
        P.Sgu = (float *)(base + o.Sgu);
        P.Sgd = (float *)(base + o.Sgd);
        P.slk = (float *)(base + o.slk);
        P.nch = G.kg / kp::CHUNK;
        P.nrel = (float *)(base + o.nrel);
        P.Wu = (float2 *)(base + o.Wu);
        P.anch = o.anch ? 1 : 0;
        P.Qt = (float *)(base + o.Qt);
        P.Wa = (float2 *)(base + o.Wa);
        P.Sdud = (float *)(base + o.Sdud);
        P.L1 = (int4 *)(base + o.L1);
        P.L1s = (int *)(base + o.L1s);
        P.L1x = (int4 *)(base + o.L1x);
        P.L3 = (int *)(base + o.L3);
        P.minnc = (float *)(base + o.minnc);
        P.tlist = (int4 *)(base + o.tlist);
        P.tcnt = (int *)(base + o.tcnt);
        P.ps4 = (float4 *)(base + o.ps4);
        P.psf = (int *)(base + o.psf);
        P.mv_pt = (int *)(base + o.mvp);
        P.mv_old = (int *)(base + o.mvo);
        P.mv_new = (int *)(base + o.mvn);
        P.srt_pt = (int *)(base + o.srtp);
        P.srt_key = (int *)(base + o.srtk);
        P.hist = (int *)(base + o.hist);
        P.cursor = (int *)(base + o.cursor);
        P.hist1 = (int *)(base + o.hist1);
        P.cursor1 = (int *)(base + o.cursor1);
        P.ctr = (unsigned long long *)(base + o.ctr);
        P.rowt = (int *)(base + o.rowt);
        P.rclosed = (unsigned *)(base + o.rclosed);
        P.stats = (long long *)(base + o.stats);
        P.iter = (int *)(base + o.iter);
        P.sink = (float *)(base + o.sink);
        P.det = det ? 1 : 0;
        P.lf = (tuning && tuning->local_filter == 1 && p.precision == KP_PREC_FP32) ? 1 : 0;
        P.nb_l1 = bits_for(P.nk1 - 1);
        P.nb_slot = bits_for(P.kg - 1);
        P.dcnt = (int *)(base + o.dcnt);
        P.doff = (int *)(base + o.doff);
        P.hist2 = (int *)(base + o.hist2);
        P.spart = (int *)(base + o.spart);
        P.pfirst = (double *)(base + o.pfirst);
        P.plast = (double *)(base + o.plast);
        KP_HIP(hipMemcpyAsync((void *)P.perm, G.perm.data(), G.perm.size() * 4, hipMemcpyHostToDevice, ctx->user));
        KP_HIP(hipMemcpyAsync((void *)P.slot_group, G.slot_group.data(), G.slot_group.size() * 4,
                              hipMemcpyHostToDevice, ctx->user));
        KP_HIP(hipMemcpyAsync((void *)P.gstart, G.gstart.data(), G.gstart.size() * 4, hipMemcpyHostToDevice,
                              ctx->user));
        KP_HIP(hipMemcpyAsync((void *)P.gsize, G.gsize.data(), G.gsize.size() * 4, hipMemcpyHostToDevice,
                              ctx->user));
        {
            std::vector<int> so((size_t)p.k, 0);
            for (size_t sl = 0; sl < G.perm.size(); ++sl)
                if (G.perm[sl] >= 0) so[(size_t)G.perm[sl]] = (int)sl;
            ctx->slot_of.push_back(std::move(so));
        }
        KP_HIP(kp::launch_prep(P, ctx->user, p.init_centroids_dev));
        KP_HIP(hipStreamSynchronize(ctx->user));   // host vectors above are reused
        ctx->P.push_back(P);
        base += o.bytes;
    }
    if (count > 1) {
        char *hdr = (char *)workspace + problem_bytes;
        kp::Batch &B = ctx->batch;
        kp::build_tables(B, ctx->P, ctx->cfg);
        B.probs = (const kp::ProbDev *)hdr;
        B.tabs = (const int *)(hdr + up((size_t)count * sizeof(kp::ProbDev), ALIGN));
        KP_HIP(hipMemcpyAsync((void *)B.probs, ctx->P.data(), (size_t)count * sizeof(kp::ProbDev),
                              hipMemcpyHostToDevice, ctx->user));
        KP_HIP(hipMemcpyAsync((void *)B.tabs, B.htabs.data(), B.htabs.size() * 4, hipMemcpyHostToDevice, ctx->user));
        KP_HIP(hipStreamSynchronize(ctx->user));
    }
    *out = guard.release();
    g_last_error.clear();
    return KP_OK;
}

static kp_status check_ctx(kp_ctx *ctx)
{
    if (!ctx) {
        set_error("ctx is NULL");
        return KP_ERR_INVALID;
    }
    if (ctx->poisoned) {
        set_error("ctx is poisoned by an earlier HIP failure");
        return KP_ERR_STATE;
    }
    return KP_OK;
}

// The stages of one iteration: those of the single problem, or each stage
// once for the whole batch.
static int iteration_calls(kp_ctx *ctx, bool dense, kp::Stage sts[kp::ST_COUNT])
{
    return ctx->count > 1 ? kp::batch_stages(ctx->P, dense, sts) : kp::iteration_stages(ctx->P[0], dense, sts);
}
static hipError_t launch_call(kp_ctx *ctx, kp::Stage st, bool dense)
{
    return ctx->count > 1 ? kp::launch_stage_batch(ctx->batch, ctx->own, st, dense, ctx->cfg)
                          : kp::launch_stage(ctx->P[0], ctx->own, st, dense, ctx->cfg);
}

// One iteration of every problem as plain launches, each stage bracketed by
// timing events when timing is on.
static hipError_t launch_all(kp_ctx *ctx, bool dense)
{
    kp::Stage sts[kp::ST_COUNT];
    const int n = iteration_calls(ctx, dense, sts);
    for (int i = 0; i < n; ++i) {
        StageTimer::Rec r;
        hipError_t e;
        const bool timed = ctx->timing && ((ctx->timed_stages >> sts[i]) & 1u);
        if (timed && (e = ctx->timer.begin(sts[i], ctx->own, r)) != hipSuccess) return e;
        if ((e = launch_call(ctx, sts[i], dense)) != hipSuccess) return e;
        if (timed && (e = ctx->timer.end(ctx->own, r)) != hipSuccess) return e;
    }
    return hipSuccess;
}

// Captures one filtered iteration of every problem into ctx->graph.  With
// timing on, each stage is captured into a graph of its own and the
// iteration graph chains them as child graphs, the timed stages between
// event-record nodes (placeholder events, re-pointed before each replay); if
// the runtime refuses that, the graph is captured in one piece and only the
// whole replay is timed.
static hipError_t capture_plain(kp_ctx *ctx)
{
    hipError_t e = hipStreamBeginCapture(ctx->own, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    kp::Stage sts[kp::ST_COUNT];
    const int n = iteration_calls(ctx, false, sts);
    for (int i = 0; i < n && e == hipSuccess; ++i) e = launch_call(ctx, sts[i], false);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(ctx->own, &g);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return e;
    }
    ctx->graph = g;
    return hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0);
}

static hipError_t capture_timed(kp_ctx *ctx, const char **where)
{
    *where = "create graph";
    hipGraph_t g = nullptr;
    hipError_t e = hipGraphCreate(&g, 0);
    if (e != hipSuccess) return e;
    ctx->graph = g;
    hipGraphNode_t last = nullptr;
    auto add_event = [&](hipEvent_t &ev) -> hipError_t {
        hipError_t r = hipEventCreate(&ev);
        if (r != hipSuccess) return r;
        ctx->cap_events.push_back(ev);
        hipGraphNode_t nd = nullptr;
        r = hipGraphAddEventRecordNode(&nd, g, last ? &last : nullptr, last ? 1 : 0, ev);
        if (r != hipSuccess) return r;
        ctx->ev_nodes.push_back(nd);
        last = nd;
        return hipSuccess;
    };
    {
        kp::Stage sts[kp::ST_COUNT];
        const int n = iteration_calls(ctx, false, sts);
        for (int i = 0; i < n; ++i) {
            hipEvent_t a = nullptr, b = nullptr;
            const bool timed = (ctx->timed_stages >> sts[i]) & 1u;
            *where = "event-record node";
            if (timed && (e = add_event(a)) != hipSuccess) return e;
            *where = "stage capture";
            if ((e = hipStreamBeginCapture(ctx->own, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
            e = launch_call(ctx, sts[i], false);
            hipGraph_t sg = nullptr;
            const hipError_t e2 = hipStreamEndCapture(ctx->own, &sg);
            if (e == hipSuccess) e = e2;
            if (e != hipSuccess) {
                if (sg) (void)hipGraphDestroy(sg);
                return e;
            }
            *where = "child graph node";
            hipGraphNode_t cn = nullptr;
            e = hipGraphAddChildGraphNode(&cn, g, last ? &last : nullptr, last ? 1 : 0, sg);
            (void)hipGraphDestroy(sg);   // the node holds its own copy
            if (e != hipSuccess) return e;
            last = cn;
            if (!timed) continue;
            *where = "event-record node";
            if ((e = add_event(b)) != hipSuccess) return e;
            ctx->ev_stage.push_back(sts[i]);
        }
    }
    *where = "instantiate";
    return hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0);
}

static hipError_t capture_iteration(kp_ctx *ctx)
{
    if (ctx->timing) {
        const char *where = "";
        const hipError_t e = capture_timed(ctx, &where);
        if (e == hipSuccess) return hipSuccess;
        // not an error of the call: the graph is captured again in one piece
        // and only whole replays are timed; the reason is kept
        set_error("stage events inside the graph unavailable (%s: %s); timing whole replays", where,
                  hipGetErrorString(e));
        (void)hipGetLastError();
        if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
        if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
        ctx->gexec = nullptr;
        ctx->graph = nullptr;
        ctx->ev_nodes.clear();
        ctx->ev_stage.clear();
    }
    return capture_plain(ctx);
}

// use_graph = 2: the iterations of one call (the dense first one included
// when the ctx has not iterated yet) captured as a single graph.  Every
// iteration's work sizes live on the device (list lengths, counters), so
// the same graph serves any later call of the same shape.
static hipError_t capture_run(kp_ctx *ctx, bool dense_first, int iters)
{
    if (ctx->rexec) (void)hipGraphExecDestroy(ctx->rexec);
    ctx->rexec = nullptr;
    hipError_t e = hipStreamBeginCapture(ctx->own, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    for (int t = 0; t < iters && e == hipSuccess; ++t) {
        const bool dense = dense_first && t == 0;
        kp::Stage sts[kp::ST_COUNT];
        const int n = iteration_calls(ctx, dense, sts);
        for (int i = 0; i < n && e == hipSuccess; ++i) e = launch_call(ctx, sts[i], dense);
    }
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(ctx->own, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&ctx->rexec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);   // the executable graph keeps what it needs
    if (e != hipSuccess) return e;
    ctx->run_iters = iters;
    ctx->run_dense = dense_first;
    return hipSuccess;
}

kp_status kp_iterate(kp_ctx *ctx, int32_t iters)
{
    kp_status st = check_ctx(ctx);
    if (st != KP_OK) return st;
    if (iters < 1) {
        set_error("iters=%d must be >= 1", iters);
        return KP_ERR_INVALID;
    }
    KP_HIP(hipEventRecord(ctx->ev_in, ctx->user));
    KP_HIP(hipStreamWaitEvent(ctx->own, ctx->ev_in, 0));
    if (ctx->plain) {
        // plain Lloyd: each iteration is the dense pass, whose update adds
        // every point to sums started from zero (cleared here on the ctx's
        // stream; this path is never captured into a graph)
        for (int i = 0; i < iters; ++i) {
            if (ctx->iters > 0)
                for (int p = 0; p < ctx->count; ++p) {
                    const kp::ProbDev &P = ctx->P[p];
                    KP_HIP(hipMemsetAsync(P.sums, 0, (size_t)P.kg * P.d * sizeof(double), ctx->own));
                    KP_HIP(hipMemsetAsync(P.cnt, 0, (size_t)P.kg * sizeof(int), ctx->own));
                }
            KP_HIP(launch_all(ctx, true));
            ++ctx->iters;
        }
        KP_HIP(hipEventRecord(ctx->ev_out, ctx->own));
        KP_HIP(hipStreamWaitEvent(ctx->user, ctx->ev_out, 0));
        return KP_OK;
    }
    if (ctx->use_graph == 2) {
        const bool dense_first = ctx->iters == 0;
        if (!ctx->rexec || ctx->run_iters != iters || ctx->run_dense != dense_first)
            KP_HIP(capture_run(ctx, dense_first, iters));
        KP_HIP(hipGraphLaunch(ctx->rexec, ctx->own));
        ctx->iters += iters;
        KP_HIP(hipEventRecord(ctx->ev_out, ctx->own));
        KP_HIP(hipStreamWaitEvent(ctx->user, ctx->ev_out, 0));
        return KP_OK;
    }
    int todo = iters;
    if (ctx->iters == 0) {
        KP_HIP(launch_all(ctx, true));
        ctx->iters = 1;
        --todo;
    }
    if (todo > 0) {
        if (ctx->use_graph) {
            if (!ctx->gexec) KP_HIP(capture_iteration(ctx));
            for (int i = 0; i < todo; ++i) {
                StageTimer::Rec r;
                std::vector<StageTimer::Rec> inner(ctx->ev_stage.size());
                if (ctx->timing) {
                    KP_HIP(ctx->timer.begin(kp::ST_COUNT, ctx->own, r));
                    for (size_t k = 0; k < inner.size(); ++k) {
                        KP_HIP(ctx->timer.take(ctx->ev_stage[k], inner[k]));
                        KP_HIP(hipGraphExecEventRecordNodeSetEvent(ctx->gexec, ctx->ev_nodes[2 * k], inner[k].a));
                        KP_HIP(hipGraphExecEventRecordNodeSetEvent(ctx->gexec, ctx->ev_nodes[2 * k + 1], inner[k].b));
                    }
                }
                KP_HIP(hipGraphLaunch(ctx->gexec, ctx->own));
                if (ctx->timing) {
                    for (auto &q : inner) ctx->timer.pending.push_back(q);
                    KP_HIP(ctx->timer.end(ctx->own, r));
                }
            }
        } else {
            for (int i = 0; i < todo; ++i) KP_HIP(launch_all(ctx, false));
        }
        ctx->iters += todo;
    }
    KP_HIP(hipEventRecord(ctx->ev_out, ctx->own));
    KP_HIP(hipStreamWaitEvent(ctx->user, ctx->ev_out, 0));
    return KP_OK;
}

kp_status kp_assign(kp_ctx *ctx, int32_t problem, int32_t *labels)
{
    kp_status st = check_ctx(ctx);
    if (st != KP_OK) return st;
    if (problem < 0 || problem >= ctx->count || !labels) {
        set_error("bad problem index %d or NULL labels", problem);
        return KP_ERR_INVALID;
    }
    if (ctx->iters == 0) {
        set_error("no iteration has run yet");
        return KP_ERR_STATE;
    }
    KP_HIP(kp::launch_labels(ctx->P[problem], ctx->user, labels));
    return KP_OK;
}

kp_status kp_centroids(kp_ctx *ctx, int32_t problem, float *c32, double *c64)
{
    kp_status st = check_ctx(ctx);
    if (st != KP_OK) return st;
    if (problem < 0 || problem >= ctx->count) {
        set_error("bad problem index %d", problem);
        return KP_ERR_INVALID;
    }
    if (!c32 && !c64) return KP_OK;
    KP_HIP(kp::launch_centroids_out(ctx->P[problem], ctx->user, c32, c64));
    return KP_OK;
}

kp_status kp_stats(kp_ctx *ctx, int32_t problem, kp_iter_stats *out, int32_t cap, int32_t *n_out)
{
    kp_status st = check_ctx(ctx);
    if (st != KP_OK) return st;
    if (problem < 0 || problem >= ctx->count || !n_out || (cap > 0 && !out) || cap < 0) {
        set_error("bad problem index %d, cap %d or NULL output", problem, cap);
        return KP_ERR_INVALID;
    }
    KP_HIP(hipStreamSynchronize(ctx->user));
    const kp::ProbDev &P = ctx->P[problem];
    int done = 0;
    KP_HIP(hipMemcpy(&done, P.iter, sizeof(int), hipMemcpyDeviceToHost));
    std::vector<long long> rec((size_t)kp::STATS_CAP * 16);
    KP_HIP(hipMemcpy(rec.data(), P.stats, rec.size() * sizeof(long long), hipMemcpyDeviceToHost));
    const int first = std::max(1, done - kp::STATS_CAP + 1);
    int w = 0;
    for (int it = first; it <= done && w < cap; ++it, ++w) {
        const long long *r = &rec[(size_t)((it - 1) % kp::STATS_CAP) * 16];
        out[w].iter = (int32_t)r[0];
        out[w].dense = (int32_t)r[1];
        out[w].point_filter_fail = r[2];
        out[w].pairs = r[3];
        out[w].distances = r[4];
        out[w].rechecks = r[5];
        out[w].moved = r[6];
        double md;
        std::memcpy(&md, &r[7], sizeof md);
        out[w].max_drift = md;
        out[w].tile_groups = r[8];
        out[w].closed = r[9];
        out[w].row_test = (int32_t)r[10];
        out[w].pad_ = 0;
    }
    *n_out = w;
    return KP_OK;
}

kp_status kp_stage_times(kp_ctx *ctx, kp_stage_time *out, int32_t cap, int32_t *n_out)
{
    kp_status st = check_ctx(ctx);
    if (st != KP_OK) return st;
    if (!n_out || cap < 0 || (cap > 0 && !out)) {
        set_error("bad cap %d or NULL output", cap);
        return KP_ERR_INVALID;
    }
    if (!ctx->timing) {
        set_error("timing is off for this ctx (kp_tuning.timing = 0)");
        return KP_ERR_STATE;
    }
    KP_HIP(hipStreamSynchronize(ctx->own));
    KP_HIP(ctx->timer.harvest());
    int w = 0;
    for (int sidx = 0; sidx < StageTimer::NSTAGE && w < cap; ++sidx) {
        if (!ctx->timer.launches[sidx]) continue;
        std::memset(out[w].name, 0, sizeof out[w].name);
        std::strncpy(out[w].name, StageTimer::name(sidx), sizeof out[w].name - 1);
        out[w].ms = ctx->timer.ms[sidx];
        out[w].launches = ctx->timer.launches[sidx];
        ++w;
    }
    *n_out = w;
    return KP_OK;
}

int32_t kp_iterations(const kp_ctx *ctx) { return ctx ? ctx->iters : -1; }

size_t kp_predict_scratch_bytes(const kp_ctx *ctx, int32_t problem, int64_t nq)
{
    if (!ctx || problem < 0 || problem >= ctx->count || nq < 0 || nq > 0x7FFFFFFFll) {
        set_error("NULL ctx, bad problem index %d or nq=%lld outside 0..2^31-1", problem, (long long)nq);
        return 0;
    }
    return kp::serve_scratch_bytes(nq, ctx->P[problem].anch != 0);
}

kp_status kp_predict(kp_ctx *ctx, int32_t problem, const float *queries, int64_t nq, int32_t *labels,
                     void *scratch, size_t scratch_bytes)
{
    kp_status st = check_ctx(ctx);
    if (st != KP_OK) return st;
    if (problem < 0 || problem >= ctx->count) {
        set_error("bad problem index %d", problem);
        return KP_ERR_INVALID;
    }
    if (nq < 0 || nq > 0x7FFFFFFFll) {
        set_error("nq=%lld outside 0..2^31-1", (long long)nq);
        return KP_ERR_INVALID;
    }
    if (nq == 0) return KP_OK;
    if (!queries || !labels || !scratch) {
        set_error("NULL queries, labels or scratch");
        return KP_ERR_INVALID;
    }
    if (((uintptr_t)queries & 15u) != 0 || ((uintptr_t)scratch & 255u) != 0) {
        set_error("queries must be 16-byte and scratch 256-byte aligned");
        return KP_ERR_INVALID;
    }
    const size_t need = kp_predict_scratch_bytes(ctx, problem, nq);
    if (scratch_bytes < need) {
        set_error("scratch of %zu bytes, %zu needed", scratch_bytes, need);
        return KP_ERR_INVALID;
    }
    KP_HIP(kp::launch_serve(ctx->P[problem], ctx->user, ctx->cfg, queries, (long long)nq, labels, scratch));
    return KP_OK;
}

kp_status kp_predict_noalloc(kp_ctx *ctx, int32_t problem, const float *queries, int64_t nq, int32_t *labels)
{
    kp_status st = check_ctx(ctx);
    if (st != KP_OK) return st;
    if (problem < 0 || problem >= ctx->count) {
        set_error("bad problem index %d", problem);
        return KP_ERR_INVALID;
    }
    if (nq < 0 || nq > kp::NOALLOC_MAX_QUERIES) {
        set_error("nq=%lld outside 0..%lld (the fixed scratch of kp_predict_noalloc)", (long long)nq,
                  (long long)kp::NOALLOC_MAX_QUERIES);
        return KP_ERR_INVALID;
    }
    if (nq == 0) return KP_OK;
    if (!queries || !labels || ((uintptr_t)queries & 15u) != 0) {
        set_error("NULL or misaligned queries, or NULL labels");
        return KP_ERR_INVALID;
    }
    void *scratch = kp::noalloc_scratch(ctx->device);
    if (!scratch) {
        set_error("no scratch address for device %d", ctx->device);
        return KP_ERR_STATE;
    }
    KP_HIP(kp::launch_serve(ctx->P[problem], ctx->user, ctx->cfg, queries, (long long)nq, labels, scratch));
    return KP_OK;
}

kp_status kp_probe_estimates(kp_ctx *ctx, int32_t problem, const float *queries, int64_t nq, int32_t anchor,
                             float *est, float *eta)
{
    kp_status st = check_ctx(ctx);
    if (st != KP_OK) return st;
    if (problem < 0 || problem >= ctx->count) {
        set_error("bad problem index %d", problem);
        return KP_ERR_INVALID;
    }
    if (nq < 0 || nq > 0x7FFFFFFFll) {
        set_error("nq=%lld outside 0..2^31-1", (long long)nq);
        return KP_ERR_INVALID;
    }
    if (ctx->P[problem].prec != KP_PREC_BF16_RECHECK) {
        set_error("problem %d is not a BF16 problem", problem);
        return KP_ERR_UNSUPPORTED;
    }
    const kp::ProbDev &P = ctx->P[problem];
    if (anchor < -1 || anchor >= P.k) {
        set_error("anchor %d outside -1..k-1", anchor);
        return KP_ERR_INVALID;
    }
    if (anchor >= 0 && !P.anch) {
        set_error("problem %d keeps no anchor tables (too many centroid slots)", problem);
        return KP_ERR_UNSUPPORTED;
    }
    if (nq == 0) return KP_OK;
    if (!queries || !est || !eta || ((uintptr_t)queries & 15u) != 0) {
        set_error("NULL or misaligned queries, NULL outputs");
        return KP_ERR_INVALID;
    }
    int slot = -1;
    if (anchor >= 0) {   // the anchor's slot (the grouping's permutation is kept on the host)
        slot = ctx->slot_of[problem][anchor];
    }
    KP_HIP(kp::launch_probe(P, ctx->user, queries, (long long)nq, slot, est, eta));
    return KP_OK;
}

kp_status kp_bounds(kp_ctx *ctx, int32_t problem, const int32_t *idx, int64_t np, float *ub, float *lbp, float *lb,
                    int32_t *groups)
{
    kp_status st = check_ctx(ctx);
    if (st != KP_OK) return st;
    if (problem < 0 || problem >= ctx->count || np < 0 || np > 0x7FFFFFFFll) {
        set_error("bad problem index %d or np=%lld outside 0..2^31-1", problem, (long long)np);
        return KP_ERR_INVALID;
    }
    if (np > 0 && (!idx || !ub || !lbp || !lb)) {
        set_error("NULL index list or outputs");
        return KP_ERR_INVALID;
    }
    if (ctx->iters == 0) {
        set_error("no iteration has run yet");
        return KP_ERR_STATE;
    }
    KP_HIP(kp::launch_bounds(ctx->P[problem], ctx->user, idx, (long long)np, ub, lbp, lb, groups));
    return KP_OK;
}

kp_status kp_autotune(const kp_problem *problems, int32_t count, void *workspace, size_t ws_bytes, void *stream,
                      int32_t iters, kp_tuning *best)
{
    if (!best || iters < 2) {
        set_error("NULL best or iters=%d < 2", iters);
        return KP_ERR_INVALID;
    }
    if (!validate(problems, count, nullptr)) return KP_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    kp_ctx *ctx = nullptr;   // for KP_HIP
    KP_HIP(hipEventCreate(&e0));
    std::unique_ptr<std::remove_pointer<hipEvent_t>::type, hipError_t (*)(hipEvent_t)> g0(e0, hipEventDestroy);
    KP_HIP(hipEventCreate(&e1));
    std::unique_ptr<std::remove_pointer<hipEvent_t>::type, hipError_t (*)(hipEvent_t)> g1(e1, hipEventDestroy);
    static const int depths[2] = {1, 3}, bpcs[3] = {8, 16, 32};
    bool any_bf = false;
    for (int i = 0; i < count; ++i) any_bf = any_bf || problems[i].precision == KP_PREC_BF16_RECHECK;
    float best_ms = -1.f;
    kp_tuning cur{};
    for (int ci = 1; ci <= (any_bf ? 2 : 1); ++ci)
        for (int di = 0; di < 2; ++di)
        for (int bi = 0; bi < 3; ++bi) {
            kp_tuning t{};
            t.bound_codes = ci;
            t.chunk_depth = depths[di];
            t.blocks_per_cu = bpcs[bi];
            t.use_graph = 1;
            kp_ctx *c = nullptr;
            kp_status st = kp_init(&c, problems, count, workspace, ws_bytes, stream, &t);
            if (st != KP_OK) return st;
            // the first call runs the dense iteration and captures the graph;
            // the timed call replays filtered iterations only
            st = kp_iterate(c, 1);
            if (st == KP_OK && hipEventRecord(e0, s) != hipSuccess) st = KP_ERR_HIP;
            if (st == KP_OK) st = kp_iterate(c, iters - 1);
            if (st == KP_OK && hipEventRecord(e1, s) != hipSuccess) st = KP_ERR_HIP;
            float ms = 0.f;
            if (st == KP_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                st = KP_ERR_HIP;
            const kp_status sd = kp_destroy(c);
            if (st != KP_OK) return st;
            if (sd != KP_OK) return sd;
            if (best_ms < 0.f || ms < best_ms) {
                best_ms = ms;
                cur = t;
            }
        }
    *best = cur;
    g_last_error.clear();
    return KP_OK;
}

kp_status kp_autotune_groups(const kp_problem *problems, int32_t count, void *workspace, size_t ws_bytes, void *stream,
                             int32_t iters, const kp_tuning *tuning, int32_t *g_out)
{
    if (!g_out || iters < 2) {
        set_error("NULL g_host or iters=%d < 2", iters);
        return KP_ERR_INVALID;
    }
    if (!validate(problems, count, tuning)) return KP_ERR_INVALID;
    if (kp_workspace_bytes(problems, count, tuning) > ws_bytes) {
        set_error("workspace of %zu bytes is smaller than the problems need", ws_bytes);
        return KP_ERR_INVALID;
    }
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    kp_ctx *ctx = nullptr;   // for KP_HIP
    KP_HIP(hipEventCreate(&e0));
    std::unique_ptr<std::remove_pointer<hipEvent_t>::type, hipError_t (*)(hipEvent_t)> h0(e0, hipEventDestroy);
    KP_HIP(hipEventCreate(&e1));
    std::unique_ptr<std::remove_pointer<hipEvent_t>::type, hipError_t (*)(hipEvent_t)> h1(e1, hipEventDestroy);
    kp_tuning t = tuning ? *tuning : kp_tuning{};
    t.timing = 0;
    t.use_graph = 1;
    // classes of equal (d, k, precision), in order of first appearance
    std::vector<std::vector<int>> classes;
    for (int i = 0; i < count; ++i) {
        bool placed = false;
        for (auto &c : classes) {
            const kp_problem &r = problems[c[0]];
            if (r.d == problems[i].d && r.k == problems[i].k && r.precision == problems[i].precision) {
                c.push_back(i);
                placed = true;
                break;
            }
        }
        if (!placed) classes.push_back({i});
    }
    for (const auto &cls : classes) {
        const kp_problem &r = problems[cls[0]];
        const int gmax = r.precision == KP_PREC_BF16_RECHECK ? std::min(r.k, 1024) : r.k;
        // candidate 0: every problem's own g; then the two rules
        std::vector<int> cand = {0};
        for (int div : {16, 10}) {
            const int g = std::max(1, std::min(gmax, (r.k + div - 1) / div));
            bool dup = true;   // the same run as candidate 0 when every problem has g already
            for (int i : cls) dup = dup && problems[i].g == g;
            for (size_t j = 1; j < cand.size(); ++j) dup = dup || cand[j] == g;
            if (!dup) cand.push_back(g);
        }
        float best_ms = -1.f;
        int best = 0;
        for (int c : cand) {
            std::vector<kp_problem> sub;
            for (int i : cls) {
                sub.push_back(problems[i]);
                if (c > 0) sub.back().g = c;
            }
            if (kp_workspace_bytes(sub.data(), (int32_t)sub.size(), &t) > ws_bytes) continue;
            kp_ctx *cx = nullptr;
            kp_status st = kp_init(&cx, sub.data(), (int32_t)sub.size(), workspace, ws_bytes, stream, &t);
            if (st != KP_OK) return st;
            st = kp_iterate(cx, 1);   // the dense iteration and the graph capture, untimed
            if (st == KP_OK && hipEventRecord(e0, s) != hipSuccess) st = KP_ERR_HIP;
            if (st == KP_OK) st = kp_iterate(cx, iters - 1);
            if (st == KP_OK && hipEventRecord(e1, s) != hipSuccess) st = KP_ERR_HIP;
            float ms = 0.f;
            if (st == KP_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                st = KP_ERR_HIP;
            const kp_status sd = kp_destroy(cx);
            if (st != KP_OK) return st;
            if (sd != KP_OK) return sd;
            if (best_ms < 0.f || ms < best_ms) {
                best_ms = ms;
                best = c;
            }
        }
        for (int i : cls) g_out[i] = best > 0 ? best : problems[i].g;
    }
    g_last_error.clear();
    return KP_OK;
}

kp_status kp_destroy(kp_ctx *ctx)
{
    if (!ctx) return KP_OK;
    kp_status st = KP_OK;
    if (ctx->user || ctx->own) {
        if (hipStreamSynchronize(ctx->user) != hipSuccess) st = KP_ERR_HIP;
        if (ctx->own && hipStreamSynchronize(ctx->own) != hipSuccess) st = KP_ERR_HIP;
    }
    release_ctx(ctx);
    if (st != KP_OK) set_error("stream synchronisation failed during kp_destroy");
    return st;
}

const char *kp_strerror(kp_status s)
{
    switch (s) {
    case KP_OK: return "success";
    case KP_ERR_INVALID: return "invalid argument";
    case KP_ERR_NOMEM: return "out of host memory";
    case KP_ERR_HIP: return "HIP runtime error";
    case KP_ERR_STATE: return "invalid state";
    case KP_ERR_UNSUPPORTED: return "unsupported configuration";
    }
    return "unknown status";
}

const char *kp_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
