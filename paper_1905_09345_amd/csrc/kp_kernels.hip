// HIP kernels (gfx950) of the filtered K-means iteration.
//
// One iteration t >= 2 of a problem runs, in stream order:
//   k_begin         clear the iteration's counters
//   k_bound_filter  point-level filter: bring each point's upper bound and
//                   point-level lower bound to iteration t and keep the points
//                   where ub < lbp fails (list L1)              [point-level filter]
//   k_assign_*      for the points of L1: tighten ub to the exact distance to
//                   the assigned centroid, retest, then test every group's
//                   lower bound against ub and compute the distances of the
//                   surviving (point, group) pairs; new assignment and bounds
//                                                  [group-level filter + distance calculator]
//   k_recheck       (BF16 mode) re-decide in FP32 direct form the points whose
//                   BF16 decision is not certain under the error bound
//   k_hist, k_scan, k_scatter, k_segsum
//                   sort the moved points by centroid and add/subtract their
//                   coordinates into FP64 centroid sums       [centroid update]
//   k_centroids     new means (FP64), their FP32 / BF16 copies, drifts
//   k_drift         per-group and global maximum drift into the FP64 rings
// Iteration 1 replaces the two filter kernels by the dense form of k_assign_*
// (every distance).  The filters follow the paper's two-level design
// (Section 1: point-level and group-level filter ahead of the distance
// calculator); the bound bookkeeping is the triangle inequality
// |d(x, c') - d(x, c)| <= ||c' - c|| applied to each centroid's drift.
#include "kp_device.h"
#include "kp_launch.h"
#include <climits>

namespace kp {

#define KP_INF __builtin_huge_valf()

// ===================================================================== prep
// BF16 shadow of the points, ||xb||^2 and the rounding residual ||x - xb||.
__global__ __launch_bounds__(256) void k_prep(ProbDev P)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P.n; i += stride) {
        const float *x = P.X + i * P.d;
        uint16_t *xb = P.Xb + i * P.ldb;
        double s = 0.0, r = 0.0;
        for (int j = 0; j < P.ldb; j += 2) {
            float v0 = j < P.d ? x[j] : 0.f;
            float v1 = j + 1 < P.d ? x[j + 1] : 0.f;
            uint16_t h0 = f2bf(v0), h1 = f2bf(v1);
            float b0 = bf2f(h0), b1 = bf2f(h1);
            *(uint32_t *)(xb + j) = (uint32_t)h0 | ((uint32_t)h1 << 16);
            s += (double)b0 * b0 + (double)b1 * b1;
            double e0 = (double)v0 - b0, e1 = (double)v1 - b1;
            r += e0 * e0 + e1 * e1;
        }
        P.xn[i] = (float)s;
        P.xr[i] = d2f_up(sqrt(r) * (1.0 + 0x1p-46));
    }
}

// ============================================================ centroid rows
// One wave per slot.  INIT: take the caller's initial centroids (original
// order).  Otherwise: c64 = sums / count (a centroid with no point keeps its
// value), then the FP32 copy, its BF16 rounding, ||c_hat||^2, ||c - c_hat||
// and the drift ||c32_new - c32_old|| (FP64, rounded up).
template <bool INIT>
__global__ __launch_bounds__(256) void k_centroids(ProbDev P, const float *init)
{
    const int lane = lane_id();
    const int nw = (int)(gridDim.x * blockDim.x / WAVE);
    const int L = P.prec ? P.ldb : P.ldc;
    for (int s = (int)((blockIdx.x * blockDim.x + threadIdx.x) / WAVE); s < P.kg; s += nw) {
        const int orig = P.perm[s];
        if (orig < 0) {
            if (INIT) {
                for (int j = lane; j < L; j += WAVE) {
                    if (j < P.ldc) P.c32[(size_t)s * P.ldc + j] = 0.f;
                    if (P.prec) P.cb[(size_t)s * P.ldb + j] = 0;
                    if (j < P.d) P.c64[(size_t)s * P.d + j] = 0.0;
                }
                if (lane == 0) {
                    P.cn[s] = KP_INF;
                    P.cr[s] = 0.f;
                    P.delta[s] = 0.0;
                }
            }
            continue;
        }
        const int cntv = INIT ? 0 : P.cnt[s];
        double dd = 0.0, q = 0.0, r = 0.0;
        for (int j = lane; j < L; j += WAVE) {
            double c64v = 0.0;
            float oldc = 0.f;
            if (j < P.d) {
                if (INIT) {
                    c64v = (double)init[(size_t)orig * P.d + j];
                } else {
                    oldc = P.c32[(size_t)s * P.ldc + j];
                    c64v = cntv > 0 ? P.sums[(size_t)s * P.d + j] / (double)cntv : P.c64[(size_t)s * P.d + j];
                }
                P.c64[(size_t)s * P.d + j] = c64v;
            }
            const float c32v = (float)c64v;
            if (j < P.ldc) P.c32[(size_t)s * P.ldc + j] = c32v;
            const uint16_t h = f2bf(c32v);
            const float hb = bf2f(h);
            if (P.prec) P.cb[(size_t)s * P.ldb + j] = h;
            const double df = (double)c32v - (double)oldc;
            dd += df * df;
            q += (double)hb * hb;
            const double e = (double)c32v - hb;
            r += e * e;
        }
        dd = wave_sum_d(dd);
        q = wave_sum_d(q);
        r = wave_sum_d(r);
        if (lane == 0) {
            P.delta[s] = INIT ? 0.0 : sqrt(dd) * (1.0 + 0x1p-46);
            P.cn[s] = (float)q;
            P.cr[s] = d2f_up(sqrt(r) * (1.0 + 0x1p-46));
        }
    }
}

// ================================================================== drifts
// Single workgroup.  After the update of iteration t: per-group maximum
// drift, global maximum, the cumulative FP64 rings at index t mod W, the
// error-bound scalars and the iteration's statistics.  first=1 at init (t=0).
__global__ __launch_bounds__(1024) void k_drift(ProbDev P, int first)
{
    __shared__ double red[1024];
    __shared__ float redf[2][1024];
    const int tid = threadIdx.x;
    const int t = first ? 0 : (*P.iter + 1);
    const int W = P.W;
    const int cur = t % W, prv = (t + W - 1) % W;
    double gmax = 0.0;
    for (int g = tid; g < P.g; g += blockDim.x) {
        double m = 0.0;
        const int s0 = P.gstart[g], ns = P.gsize[g];
        for (int r = 0; r < ns; ++r) m = fmax(m, P.delta[s0 + r]);
        P.Sg[(size_t)cur * P.g + g] = (t == 0 ? 0.0 : P.Sg[(size_t)prv * P.g + g]) + m;
        gmax = fmax(gmax, m);
    }
    float bmax = 0.f, rmax = 0.f;
    for (int s = tid; s < P.kg; s += blockDim.x) {
        P.Sc[(size_t)cur * P.kg + s] = (t == 0 ? 0.0 : P.Sc[(size_t)prv * P.kg + s]) + P.delta[s];
        if (P.perm[s] >= 0) {
            bmax = fmaxf(bmax, P.cn[s]);
            rmax = fmaxf(rmax, P.cr[s]);
        }
    }
    red[tid] = gmax;
    redf[0][tid] = bmax;
    redf[1][tid] = rmax;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (tid < o) {
            red[tid] = fmax(red[tid], red[tid + o]);
            redf[0][tid] = fmaxf(redf[0][tid], redf[0][tid + o]);
            redf[1][tid] = fmaxf(redf[1][tid], redf[1][tid + o]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        P.Sd[cur] = (t == 0 ? 0.0 : P.Sd[prv]) + red[0];
        P.scal[0] = d2f_up(sqrt((double)redf[0][0]) * (1.0 + 0x1p-46));
        P.scal[1] = redf[1][0];
        if (!first) {
            long long *rec = P.stats + (size_t)((t - 1) % STATS_CAP) * 8;
            rec[0] = t;
            rec[1] = (long long)P.ctr[CTR_DENSE];
            rec[2] = (long long)P.ctr[CTR_L1];
            rec[3] = (long long)P.ctr[CTR_PAIRS];
            rec[4] = (long long)P.ctr[CTR_DIST];
            rec[5] = (long long)P.ctr[CTR_L3];
            rec[6] = (long long)P.ctr[CTR_MOVED];
            rec[7] = 0;
            *P.iter = t;
        }
    }
}

// ================================================================= begin
__global__ void k_begin(ProbDev P, int dense)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid < NCTR) P.ctr[tid] = (tid == CTR_DENSE) ? (unsigned long long)dense : 0ull;
    for (int s = tid; s <= P.kg; s += gridDim.x * blockDim.x) P.hist[s] = 0;
}

// ========================================================== bound filter
// Point-level filter.  ub_eff = ub + drift of the own centroid since tx,
// lbp_eff = lbp - largest drift of any centroid since tx.  A point is kept
// (list L1) unless ub_eff < lbp_eff; points whose stamp is W-1 iterations old
// are kept as well so that their stored bounds are refreshed before the
// drift ring wraps.
__global__ __launch_bounds__(256) void k_bound_filter(ProbDev P)
{
    const int t = *P.iter + 1;
    const int W = P.W;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < P.n; base += stride) {
        const int64_t i = base + threadIdx.x;
        bool keep = false;
        if (i < P.n) {
            const PointState s = P.st[i];
            const double ub = up_eff(s.ub, drift_between(P.Sc, P.kg, s.a, t, s.tx, W));
            const double lp = lo_eff(s.lbp, drift_between(P.Sd, 1, 0, t, s.tx, W));
            keep = !(ub < lp) || (t - s.tx >= W - 1);
        }
        const long long pos = wave_append(&P.ctr[CTR_L1], keep);
        if (pos >= 0) P.L1[pos] = (int)i;
    }
}

// ===================================================== FP32 direct distance
// Squared distance in the direct form with accumulator i mod 4 (see
// eps2_direct).  x has `DMAX` registers, zero beyond d; c is a row padded
// with zeros to ldc (a multiple of 4).  The same order is used everywhere a
// direct distance is computed, so equal inputs give equal results.
template <int DMAX>
__device__ __forceinline__ float direct_d2(const float (&x)[DMAX], const float *__restrict__ c, int ldc)
{
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
#pragma unroll
    for (int i = 0; i < DMAX; i += 4) {
        if (i < ldc) {
            const float4 cv = *(const float4 *)(c + i);
            const float t0 = x[i] - cv.x, t1 = x[i + 1] - cv.y, t2 = x[i + 2] - cv.z, t3 = x[i + 3] - cv.w;
            a0 = fmaf(t0, t0, a0);
            a1 = fmaf(t1, t1, a1);
            a2 = fmaf(t2, t2, a2);
            a3 = fmaf(t3, t3, a3);
        }
    }
    return (a0 + a1) + (a2 + a3);
}

// Same arithmetic with both rows read from memory (x unpadded, length d).
__device__ __forceinline__ float direct_d2_mem(const float *__restrict__ x, const float *__restrict__ c, int d)
{
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    int i = 0;
    if ((d & 3) == 0) {
        for (; i < d; i += 4) {
            const float4 xv = *(const float4 *)(x + i);
            const float4 cv = *(const float4 *)(c + i);
            const float t0 = xv.x - cv.x, t1 = xv.y - cv.y, t2 = xv.z - cv.z, t3 = xv.w - cv.w;
            a0 = fmaf(t0, t0, a0);
            a1 = fmaf(t1, t1, a1);
            a2 = fmaf(t2, t2, a2);
            a3 = fmaf(t3, t3, a3);
        }
    } else {
        for (; i < d; i += 4) {
            const float t0 = x[i] - c[i];
            const float t1 = (i + 1 < d ? x[i + 1] : 0.f) - c[i + 1];
            const float t2 = (i + 2 < d ? x[i + 2] : 0.f) - c[i + 2];
            const float t3 = (i + 3 < d ? x[i + 3] : 0.f) - c[i + 3];
            a0 = fmaf(t0, t0, a0);
            a1 = fmaf(t1, t1, a1);
            a2 = fmaf(t2, t2, a2);
            a3 = fmaf(t3, t3, a3);
        }
    }
    return (a0 + a1) + (a2 + a3);
}

// Is (v, slot sa) before (w, slot sb) in (distance, original index) order?
__device__ __forceinline__ bool before(const ProbDev &P, float v, int sa, float w, int sb)
{
    if (v < w) return true;
    if (v > w || sb < 0) return sb < 0 && v == w;
    return P.perm[sa] < P.perm[sb];
}

// Per-tile bookkeeping shared by both engines ---------------------------------
struct TileState {
    int pid;          // point id (-1: lane empty)
    bool active;      // still needs the group stage
    int a, ga, tx;    // old slot, its group, stamp (survivor mode)
    float d2a;        // direct d^2 to the old centroid
    float ubt;        // tightened upper bound on d(x, c_a)
    bool a_sep;       // old centroid tracked separately (its group did not survive)
    float lbe_a;      // effective lower bound of the old group
};

// Load the tile's points, tighten ub, retest the point-level bound.  Points
// that pass after tightening get their stored ub replaced (stamp unchanged:
// the stored value is shifted back by the drift accumulated since tx).
__device__ __forceinline__ TileState tile_begin(const ProbDev &P, bool dense, long long tl, long long count,
                                                int t, double eps2)
{
    TileState ts;
    const int lane = lane_id();
    const long long idx = tl * WAVE + lane;
    ts.pid = -1;
    ts.active = false;
    ts.a = -1;
    ts.ga = -1;
    ts.tx = t;
    ts.d2a = KP_INF;
    ts.ubt = KP_INF;
    ts.a_sep = false;
    ts.lbe_a = KP_INF;
    if (idx < count) ts.pid = dense ? (int)idx : P.L1[idx];
    if (ts.pid < 0) return ts;
    ts.active = true;
    if (dense) return ts;
    const PointState s = P.st[ts.pid];
    ts.a = s.a;
    ts.tx = s.tx;
    ts.ga = P.slot_group[s.a];
    const int W = P.W;
    const double lp = lo_eff(s.lbp, drift_between(P.Sd, 1, 0, t, s.tx, W));
    ts.d2a = direct_d2_mem(P.X + (size_t)ts.pid * P.d, P.c32 + (size_t)s.a * P.ldc, P.d);
    ts.ubt = dist_hi(ts.d2a, eps2);
    if ((double)ts.ubt < lp && (t - s.tx) < W - 1) {
        const double shifted = (double)ts.ubt - drift_between_dn(P.Sc, P.kg, s.a, t, s.tx, W);
        P.st[ts.pid].ub = d2f_up(shifted + fabs(shifted) * 0x1p-50);
        ts.active = false;
        return ts;
    }
    const float lbv = P.lb[(size_t)ts.pid * P.gs + ts.ga];
    ts.lbe_a = d2f_dn(lo_eff(lbv, drift_between(P.Sg, P.g, ts.ga, t, s.tx, W)));
    ts.a_sep = (ts.ubt < ts.lbe_a);
    return ts;
}

// ============================================== FP32 engine: lane per point
// x lives in registers; the centroid rows of a group are uniform across the
// wave (scalar loads).  No recheck is needed: decisions are taken on direct
// FP32 values whose relative error (eps2_direct) is far below the near-tie
// band, and every bound carries that error.
template <int DMAX, bool DENSE>
__global__ __launch_bounds__(256) void k_assign_f32(ProbDev P)
{
    const int lane = lane_id();
    const int wpb = blockDim.x / WAVE;
    const int t = *P.iter + 1;
    const int W = P.W;
    const double eps2 = eps2_direct(P.d);
    const long long count = DENSE ? P.n : (long long)P.ctr[CTR_L1];
    const long long ntiles = (count + WAVE - 1) / WAVE;
    unsigned long long n_pairs = 0, n_dist = 0;
    for (long long tl = (long long)blockIdx.x * wpb + threadIdx.x / WAVE; tl < ntiles;
         tl += (long long)gridDim.x * wpb) {
        TileState ts = tile_begin(P, DENSE, tl, count, t, eps2);
        const bool act = ts.active;
        if (__ballot(act) == 0ull) continue;
        float x[DMAX];
#pragma unroll
        for (int i = 0; i < DMAX; ++i) x[i] = 0.f;
        if (act) {
            const float *xr = P.X + (size_t)ts.pid * P.d;
#pragma unroll
            for (int i = 0; i < DMAX; ++i)
                if (i < P.d) x[i] = xr[i];
        }
        // running best over everything examined (old centroid included when
        // its group did not survive)
        float bd = KP_INF, sec = KP_INF, bm2 = KP_INF, minnc = KP_INF;
        int bs = -1, bg = -1;
        if (!DENSE && ts.a_sep) {
            bd = ts.d2a;
            bs = ts.a;
            bg = -1;   // not from a computed group
        }
        float *lbrow = act ? P.lb + (size_t)ts.pid * P.gs : nullptr;
        for (int g4 = 0; g4 < P.g; g4 += 4) {
            float4 lbq = make_float4(0.f, 0.f, 0.f, 0.f);
            if (!DENSE && act) lbq = *(const float4 *)(lbrow + g4);
            float outv[4] = {KP_INF, KP_INF, KP_INF, KP_INF};
            const float lbin[4] = {lbq.x, lbq.y, lbq.z, lbq.w};
#pragma unroll
            for (int gg = 0; gg < 4; ++gg) {
                const int g = g4 + gg;
                if (g >= P.g) break;
                bool cand;
                float lbe = KP_INF;
                if (DENSE) {
                    cand = act;
                } else {
                    if (act) lbe = d2f_dn(lo_eff(lbin[gg], drift_between(P.Sg, P.g, g, t, ts.tx, W)));
                    cand = act && !(ts.ubt < lbe);
                }
                const unsigned long long m = __ballot(cand);
                float gm1 = KP_INF, gm2 = KP_INF;
                int gs1 = -1;
                if (m) {
                    const int s0 = P.gstart[g], ns = P.gsize[g];
                    for (int r = 0; r < ns; ++r) {
                        const float v = direct_d2<DMAX>(x, P.c32 + (size_t)(s0 + r) * P.ldc, P.ldc);
                        if (v < gm1) {
                            gm2 = gm1;
                            gm1 = v;
                            gs1 = s0 + r;
                        } else {
                            gm2 = fminf(gm2, v);
                        }
                    }
                    n_pairs += (unsigned long long)__popcll(m);
                    n_dist += (unsigned long long)__popcll(m) * (unsigned long long)ns;
                }
                if (cand) {
                    outv[gg] = dist_lo(gm1, eps2);
                    if (before(P, gm1, gs1, bd, bs)) {
                        sec = fminf(bd, gm2);
                        bd = gm1;
                        bs = gs1;
                        bg = g;
                        bm2 = gm2;
                    } else {
                        sec = fminf(sec, gm1);
                    }
                } else if (act) {
                    outv[gg] = lbe;
                    minnc = fminf(minnc, lbe);
                }
            }
            if (act) *(float4 *)(lbrow + g4) = make_float4(outv[0], outv[1], outv[2], outv[3]);
        }
        bool moved = false;
        int oldslot = DENSE ? -1 : ts.a;
        if (act) {
            if (bg >= 0) lbrow[bg] = dist_lo(bm2, eps2);
            float lbp = fminf(dist_lo(sec, eps2), minnc);
            if (!DENSE && ts.a_sep && bs != ts.a) {
                const float v = fminf(ts.lbe_a, dist_lo(ts.d2a, eps2));
                lbrow[ts.ga] = v;
                lbp = fminf(lbp, v);
            }
            PointState ns;
            ns.a = bs;
            ns.ub = dist_hi(bd, eps2);
            ns.lbp = lbp;
            ns.tx = t;
            P.st[ts.pid] = ns;
            moved = (bs != oldslot);
        }
        const long long pos = wave_append(&P.ctr[CTR_MOVED], moved);
        if (pos >= 0) {
            P.mv_pt[pos] = ts.pid;
            P.mv_old[pos] = oldslot;
            P.mv_new[pos] = bs;
        }
    }
    if (lane == 0 && n_pairs) {
        atomicAdd(&P.ctr[CTR_PAIRS], n_pairs);
        atomicAdd(&P.ctr[CTR_DIST], n_dist);
    }
}

// ============================================== BF16 engine: MFMA per group
// A wave owns 64 points (lane l <-> point l of the tile).  For one 16-slot
// chunk of a group, v_mfma_f32_16x16x32_bf16 with A = the 16 centroids and
// B = 16 points gives lane l the products of point (l & 15) of the block
// with centroids 4*(l >> 4) .. +3 of the chunk.  Four blocks cover the 64
// points; a transposing reduction over the four lane groups leaves lane l
// with the (best, slot, second) of its own point for the chunk.
__device__ __forceinline__ Best3 best_of4(const float v[4], int slot0)
{
    Best3 b;
    b.m1 = v[0];
    b.s1 = slot0;
    b.m2 = KP_INF;
#pragma unroll
    for (int r = 1; r < 4; ++r) {
        if (v[r] < b.m1) {
            b.m2 = b.m1;
            b.m1 = v[r];
            b.s1 = slot0 + r;
        } else {
            b.m2 = fminf(b.m2, v[r]);
        }
    }
    return b;
}

// T[blk] holds, for point (16 blk + (l & 15)), the result over centroid rows
// 4q .. 4q+3 (q = l >> 4).  Returns the merge over q of T[q'] for block q,
// i.e. the result of point l.
__device__ __forceinline__ Best3 transpose_reduce(const Best3 (&T)[4])
{
    const int q = lane_id() >> 4;
    const bool hi = q >= 2;
    Best3 U[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const Best3 keep = hi ? T[2 + j] : T[j];
        const Best3 send = hi ? T[j] : T[2 + j];
        U[j] = merge3(keep, shfl_xor3(send, 32));
    }
    const bool odd = q & 1;
    const Best3 keep = odd ? U[1] : U[0];
    const Best3 send = odd ? U[0] : U[1];
    return merge3(keep, shfl_xor3(send, 16));
}

template <int KS, bool DENSE>
__global__ __launch_bounds__(256) void k_assign_bf16(ProbDev P)
{
    const int lane = lane_id();
    const int wpb = blockDim.x / WAVE;
    const int t = *P.iter + 1;
    const int W = P.W;
    const double eps2 = eps2_direct(P.d);
    const float bmax = P.scal[0], rcmax = P.scal[1];
    const long long count = DENSE ? P.n : (long long)P.ctr[CTR_L1];
    const long long ntiles = (count + WAVE - 1) / WAVE;
    const int col = lane & 15, quad = lane >> 4;
    unsigned long long n_pairs = 0, n_dist = 0;
    for (long long tl = (long long)blockIdx.x * wpb + threadIdx.x / WAVE; tl < ntiles;
         tl += (long long)gridDim.x * wpb) {
        TileState ts = tile_begin(P, DENSE, tl, count, t, eps2);
        const bool act = ts.active;
        const unsigned long long amask = __ballot(act);
        if (amask == 0ull) continue;
        // B fragments: point 16*blk + col, k = ks*32 + 8*quad .. +7
        bf16x8 bx[4][KS];
        float xnB[4];
#pragma unroll
        for (int blk = 0; blk < 4; ++blk) {
            const int src = 16 * blk + col;
            const int p = __shfl(ts.pid, src);
            const bool ok = (amask >> src) & 1ull;
            xnB[blk] = ok ? P.xn[p] : 0.f;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                if (ok) {
                    bx[blk][ks] = *(const bf16x8 *)(P.Xb + (size_t)p * P.ldb + ks * 32 + 8 * quad);
                } else {
                    bx[blk][ks] = bf16x8{};
                }
            }
        }
        double eta = 0.0, rho = 0.0;
        if (act) {
            eta = mfma_eta(P.xn[ts.pid], bmax, P.ldb);
            rho = (double)P.xr[ts.pid] + (double)rcmax;
        }
        float mb = KP_INF, msec = KP_INF, mbm2 = KP_INF, minnc = KP_INF;
        int ms = -1, mbg = -1;
        float *lbrow = act ? P.lb + (size_t)ts.pid * P.gs : nullptr;
        for (int g4 = 0; g4 < P.g; g4 += 4) {
            float4 lbq = make_float4(0.f, 0.f, 0.f, 0.f);
            if (!DENSE && act) lbq = *(const float4 *)(lbrow + g4);
            float outv[4] = {KP_INF, KP_INF, KP_INF, KP_INF};
            const float lbin[4] = {lbq.x, lbq.y, lbq.z, lbq.w};
#pragma unroll 1
            for (int gg = 0; gg < 4; ++gg) {
                const int g = g4 + gg;
                if (g >= P.g) break;
                bool cand;
                float lbe = KP_INF;
                if (DENSE) {
                    cand = act;
                } else {
                    if (act) lbe = d2f_dn(lo_eff(lbin[gg], drift_between(P.Sg, P.g, g, t, ts.tx, W)));
                    cand = act && !(ts.ubt < lbe);
                }
                const unsigned long long m = __ballot(cand);
                Best3 gb = {KP_INF, INT_MAX, KP_INF};
                if (m) {
                    const int s0 = P.gstart[g], ns = P.gsize[g];
                    for (int c0 = 0; c0 < ns; c0 += CHUNK) {
                        const int slot0 = s0 + c0;
                        bf16x8 af[KS];
#pragma unroll
                        for (int ks = 0; ks < KS; ++ks)
                            af[ks] = *(const bf16x8 *)(P.cb + (size_t)(slot0 + col) * P.ldb + ks * 32 + 8 * quad);
                        const float4 cn4 = *(const float4 *)(P.cn + slot0 + 4 * quad);
                        const float cnv[4] = {cn4.x, cn4.y, cn4.z, cn4.w};
                        Best3 T[4];
#pragma unroll
                        for (int blk = 0; blk < 4; ++blk) {
                            if ((m >> (16 * blk)) & 0xFFFFull) {
                                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                                for (int ks = 0; ks < KS; ++ks)
                                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[ks], bx[blk][ks], acc, 0, 0, 0);
                                float v[4];
#pragma unroll
                                for (int r = 0; r < 4; ++r) v[r] = fmaf(-2.f, acc[r], xnB[blk] + cnv[r]);
                                T[blk] = best_of4(v, slot0 + 4 * quad);
                            } else {
                                T[blk].m1 = KP_INF;
                                T[blk].s1 = INT_MAX;
                                T[blk].m2 = KP_INF;
                            }
                        }
                        gb = merge3(gb, transpose_reduce(T));
                    }
                    n_pairs += (unsigned long long)__popcll(m);
                    n_dist += (unsigned long long)__popcll(m) * (unsigned long long)ns;
                }
                if (cand) {
                    outv[gg] = mfma_lo(gb.m1, eta, rho);
                    if (before(P, gb.m1, gb.s1, mb, ms)) {
                        msec = fminf(mb, gb.m2);
                        mb = gb.m1;
                        ms = gb.s1;
                        mbg = g;
                        mbm2 = gb.m2;
                    } else {
                        msec = fminf(msec, gb.m1);
                    }
                } else if (act) {
                    outv[gg] = lbe;
                    minnc = fminf(minnc, lbe);
                }
            }
            if (act) *(float4 *)(lbrow + g4) = make_float4(outv[0], outv[1], outv[2], outv[3]);
        }
        // decision under the error bound
        const int oldslot = DENSE ? -1 : ts.a;
        bool moved = false, amb = false;
        int win = -1;
        float umin = KP_INF;
        if (act) {
            const float Lb = mfma_lo(mb, eta, rho), Ub = mb < KP_INF ? mfma_hi(mb, eta, rho) : KP_INF;
            const float Ls = mfma_lo(msec, eta, rho);
            const bool a_sep = !DENSE && ts.a_sep;
            float La = KP_INF;
            if (a_sep) {
                La = dist_lo(ts.d2a, eps2);
                if (ts.ubt < Lb) {
                    win = ts.a;   // old centroid certainly nearest
                } else if (Ub < La && Ub < Ls) {
                    win = ms;
                } else {
                    amb = true;
                    umin = fminf(Ub, ts.ubt);
                }
            } else {
                if (Ub < Ls) win = ms;
                else {
                    amb = true;
                    umin = Ub;
                }
            }
            if (!amb) {
                PointState nsv;
                nsv.a = win;
                nsv.tx = t;
                if (win == ts.a && a_sep) {
                    nsv.ub = ts.ubt;
                    nsv.lbp = fminf(minnc, Lb);
                } else {
                    lbrow[mbg] = mfma_lo(mbm2, eta, rho);
                    nsv.ub = Ub;
                    float lbp = fminf(minnc, Ls);
                    if (a_sep) {
                        const float v = fminf(ts.lbe_a, La);
                        lbrow[ts.ga] = v;
                        lbp = fminf(lbp, v);
                    }
                    nsv.lbp = lbp;
                }
                P.st[ts.pid] = nsv;
                moved = (win != oldslot);
            }
        }
        const long long pos = wave_append(&P.ctr[CTR_MOVED], moved);
        if (pos >= 0) {
            P.mv_pt[pos] = ts.pid;
            P.mv_old[pos] = oldslot;
            P.mv_new[pos] = win;
        }
        const long long p3 = wave_append(&P.ctr[CTR_L3], amb);
        if (p3 >= 0) {
            const bool a_sep = !DENSE && ts.a_sep;
            P.L3[p3] = make_int4(ts.pid, oldslot, __float_as_int(umin), a_sep ? 1 : 0);
        }
    }
    if (lane == 0 && n_pairs) {
        atomicAdd(&P.ctr[CTR_PAIRS], n_pairs);
        atomicAdd(&P.ctr[CTR_DIST], n_dist);
    }
}

// ================================================================ recheck
// One wave per uncertain point.  Candidates: every group whose (provisional)
// lower bound is <= U*, an upper bound on the point's true nearest distance,
// plus the old centroid when it was tracked separately.  Every other centroid
// is provably farther than the nearest one.  Distances are recomputed in FP32
// direct form; lane (r, q) = (lane >> 2, lane & 3) sums coordinates
// i = q mod 4 of member r, so the value equals direct_d2 bit for bit.
constexpr int RECHECK_MAXG = 1024;

__device__ __forceinline__ float direct_lane(const float *__restrict__ x, const float *__restrict__ c, int d, int q)
{
    float acc = 0.f;
    for (int i = q; i < d; i += 4) {
        const float t0 = x[i] - c[i];
        acc = fmaf(t0, t0, acc);
    }
    float v = acc + __shfl_xor(acc, 1);
    return v + __shfl_xor(v, 2);
}

__global__ __launch_bounds__(256) void k_recheck(ProbDev P)
{
    __shared__ int rg[4][RECHECK_MAXG];
    __shared__ float rm1[4][RECHECK_MAXG], rm2[4][RECHECK_MAXG];
    const int lane = lane_id();
    const int wv = threadIdx.x / WAVE;
    const int t = *P.iter + 1;
    const double eps2 = eps2_direct(P.d);
    const long long nL3 = (long long)P.ctr[CTR_L3];
    const long long nw = (long long)gridDim.x * (blockDim.x / WAVE);
    const int r = lane >> 2, q = lane & 3;
    for (long long e = (long long)blockIdx.x * (blockDim.x / WAVE) + wv; e < nL3; e += nw) {
        const int4 ent = P.L3[e];
        const int pid = ent.x, olda = ent.y;
        const float umin = __int_as_float(ent.z);
        const bool a_sep = ent.w & 1;
        const float *xrow = P.X + (size_t)pid * P.d;
        float *lbrow = P.lb + (size_t)pid * P.gs;
        float minnr = KP_INF;
        int nR = 0;
        for (int g0 = 0; g0 < P.g; g0 += WAVE) {
            const int g = g0 + lane;
            const float v = g < P.g ? lbrow[g] : KP_INF;
            const bool inR = g < P.g && v <= umin;
            if (!inR) minnr = fminf(minnr, v);
            const unsigned long long m = __ballot(inR);
            if (inR) rg[wv][nR + __popcll(m & ((1ull << lane) - 1ull))] = g;
            nR += __popcll(m);
        }
        minnr = wave_min(minnr);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        float bd = KP_INF;
        int bs = -1, bgi = -1;
        for (int i = 0; i < nR; ++i) {
            const int g = rg[wv][i];
            const int s0 = P.gstart[g], ns = P.gsize[g];
            Best3 gb = {KP_INF, INT_MAX, KP_INF};
            for (int c0 = 0; c0 < ns; c0 += 16) {
                const int mr = c0 + r;
                const bool ok = mr < ns;
                const int slot = s0 + (ok ? mr : 0);
                const float v = direct_lane(xrow, P.c32 + (size_t)slot * P.ldc, P.d, q);
                Best3 c;
                c.m1 = ok ? v : KP_INF;
                c.s1 = ok ? s0 + mr : INT_MAX;
                c.m2 = KP_INF;
#pragma unroll
                for (int o = 4; o < WAVE; o <<= 1) c = merge3(c, shfl_xor3(c, o));
                gb = merge3(gb, c);
            }
            if (lane == 0) {
                rm1[wv][i] = gb.m1;
                rm2[wv][i] = gb.m2;
            }
            if (before(P, gb.m1, gb.s1, bd, bs)) {
                bd = gb.m1;
                bs = gb.s1;
                bgi = i;
            }
        }
        float d2a = KP_INF;
        if (a_sep && olda >= 0) {
            d2a = __shfl(direct_lane(xrow, P.c32 + (size_t)olda * P.ldc, P.d, q), 0);
            if (before(P, d2a, olda, bd, bs)) {
                bd = d2a;
                bs = olda;
                bgi = -1;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        float minr = KP_INF;
        for (int i = lane; i < nR; i += WAVE) {
            const float v = dist_lo(i == bgi ? rm2[wv][i] : rm1[wv][i], eps2);
            lbrow[rg[wv][i]] = v;
            minr = fminf(minr, v);
        }
        float lbp = fminf(minnr, wave_min(minr));
        if (a_sep && olda >= 0 && bs != olda) {
            const int ga = P.slot_group[olda];
            const float v = fminf(lbrow[ga], dist_lo(d2a, eps2));
            if (lane == 0) lbrow[ga] = v;
            lbp = fminf(lbp, v);
        }
        if (lane == 0) {
            PointState nsv;
            nsv.a = bs;
            nsv.ub = dist_hi(bd, eps2);
            nsv.lbp = lbp;
            nsv.tx = t;
            P.st[pid] = nsv;
            if (bs != olda) {
                const unsigned long long pos = atomicAdd(&P.ctr[CTR_MOVED], 1ull);
                P.mv_pt[pos] = pid;
                P.mv_old[pos] = olda;
                P.mv_new[pos] = bs;
            }
        }
    }
}

// ========================================================= centroid update
// Entries: e < M adds point mv_pt[e] to slot mv_new[e]; M <= e < 2M subtracts
// point mv_pt[e-M] from slot mv_old[e-M] (skipped when there was none).
constexpr int HIST_LDS = 8192;

__device__ __forceinline__ int entry_key(const ProbDev &P, long long e, long long M)
{
    return e < M ? P.mv_new[e] : P.mv_old[e - M];
}

__global__ __launch_bounds__(256) void k_hist(ProbDev P)
{
    __shared__ int h[HIST_LDS];
    const long long M = (long long)P.ctr[CTR_MOVED];
    const long long E = 2 * M;
    const bool lds = P.kg <= HIST_LDS;
    if (lds)
        for (int i = threadIdx.x; i < P.kg; i += blockDim.x) h[i] = 0;
    __syncthreads();
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < E;
         e += (long long)gridDim.x * blockDim.x) {
        const int key = entry_key(P, e, M);
        if (key < 0) continue;
        if (lds) atomicAdd(&h[key], 1);
        else atomicAdd(&P.hist[key], 1);
    }
    __syncthreads();
    if (lds)
        for (int i = threadIdx.x; i < P.kg; i += blockDim.x)
            if (h[i]) atomicAdd(&P.hist[i], h[i]);
}

// Exclusive scan of hist into cursor (single workgroup of 1024).
__global__ __launch_bounds__(1024) void k_scan(ProbDev P)
{
    __shared__ int part[1024];
    const int tid = threadIdx.x;
    const int n = P.kg;
    const int per = (n + 1023) / 1024;
    const int b = tid * per, e = min(n, b + per);
    int s = 0;
    for (int i = b; i < e; ++i) s += P.hist[i];
    part[tid] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int v = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int run = part[tid] - s;
    for (int i = b; i < e; ++i) {
        P.cursor[i] = run;
        run += P.hist[i];
    }
}

__global__ __launch_bounds__(256) void k_scatter(ProbDev P)
{
    __shared__ int h[HIST_LDS];
    __shared__ int base[HIST_LDS];
    const long long M = (long long)P.ctr[CTR_MOVED];
    const long long E = 2 * M;
    const bool lds = P.kg <= HIST_LDS;
    const long long b0 = E * blockIdx.x / gridDim.x, b1 = E * (blockIdx.x + 1) / gridDim.x;
    if (!lds) {
        for (long long e = b0 + threadIdx.x; e < b1; e += blockDim.x) {
            const int key = entry_key(P, e, M);
            if (key < 0) continue;
            const int pos = atomicAdd(&P.cursor[key], 1);
            const int pid = P.mv_pt[e < M ? e : e - M];
            P.srt_pt[pos] = e < M ? pid : (int)((unsigned)pid | 0x80000000u);
            P.srt_key[pos] = key;
        }
        return;
    }
    if (b0 >= b1) return;   // uniform per block
    for (int i = threadIdx.x; i < P.kg; i += blockDim.x) h[i] = 0;
    __syncthreads();
    for (long long e = b0 + threadIdx.x; e < b1; e += blockDim.x) {
        const int key = entry_key(P, e, M);
        if (key >= 0) atomicAdd(&h[key], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < P.kg; i += blockDim.x) {
        base[i] = h[i] ? atomicAdd(&P.cursor[i], h[i]) : 0;
        h[i] = 0;
    }
    __syncthreads();
    for (long long e = b0 + threadIdx.x; e < b1; e += blockDim.x) {
        const int key = entry_key(P, e, M);
        if (key < 0) continue;
        const int pos = base[key] + atomicAdd(&h[key], 1);
        const int pid = P.mv_pt[e < M ? e : e - M];
        P.srt_pt[pos] = e < M ? pid : (int)((unsigned)pid | 0x80000000u);
        P.srt_key[pos] = key;
    }
}

// One wave per run of 64 sorted entries; lanes over coordinates.  Sums are
// FP64; a change of key flushes the run with FP64 atomics.
template <int DCH>
__global__ __launch_bounds__(256) void k_segsum(ProbDev P)
{
    const int lane = lane_id();
    const long long M = (long long)P.ctr[CTR_MOVED];
    long long E = 0;
    // number of sorted entries = sum of hist
    // (entries with no old slot were skipped)
    E = 2 * M;   // upper bound; the real count is cursor[kg-1] after scatter
    const long long used = (long long)P.cursor[P.kg - 1];
    E = used < E ? used : E;
    const long long nchunks = (E + WAVE - 1) / WAVE;
    const long long nw = (long long)gridDim.x * (blockDim.x / WAVE);
    for (long long c = (long long)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE; c < nchunks; c += nw) {
        const long long p0 = c * WAVE, p1 = (p0 + WAVE < E) ? p0 + WAVE : E;
        double acc[DCH];
#pragma unroll
        for (int j = 0; j < DCH; ++j) acc[j] = 0.0;
        int cacc = 0;
        int cur = P.srt_key[p0];
        for (long long p = p0; p < p1; ++p) {
            const int key = P.srt_key[p];
            const int v = P.srt_pt[p];
            if (key != cur) {
#pragma unroll
                for (int j = 0; j < DCH; ++j) {
                    const int dim = lane + WAVE * j;
                    if (dim < P.d) atomicAdd(&P.sums[(size_t)cur * P.d + dim], acc[j]);
                    acc[j] = 0.0;
                }
                if (lane == 0) atomicAdd(&P.cnt[cur], cacc);
                cacc = 0;
                cur = key;
            }
            const int pid = v & 0x7FFFFFFF;
            const bool neg = v < 0;
            const float *xr = P.X + (size_t)pid * P.d;
#pragma unroll
            for (int j = 0; j < DCH; ++j) {
                const int dim = lane + WAVE * j;
                if (dim < P.d) {
                    const double xv = (double)xr[dim];
                    acc[j] += neg ? -xv : xv;
                }
            }
            cacc += neg ? -1 : 1;
        }
#pragma unroll
        for (int j = 0; j < DCH; ++j) {
            const int dim = lane + WAVE * j;
            if (dim < P.d) atomicAdd(&P.sums[(size_t)cur * P.d + dim], acc[j]);
        }
        if (lane == 0) atomicAdd(&P.cnt[cur], cacc);
    }
}

// ================================================================ outputs
__global__ void k_labels(ProbDev P, int *out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P.n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = P.perm[P.st[i].a];
}

__global__ void k_centroids_out(ProbDev P, float *c32, double *c64)
{
    const int64_t total = (int64_t)P.kg * P.d;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int s = (int)(i / P.d), j = (int)(i % P.d);
        const int o = P.perm[s];
        if (o < 0) continue;
        if (c32) c32[(size_t)o * P.d + j] = P.c32[(size_t)s * P.ldc + j];
        if (c64) c64[(size_t)o * P.d + j] = P.c64[(size_t)s * P.d + j];
    }
}

// ================================================================ launches
static inline int cap_grid(long long want, int cap)
{
    if (want < 1) want = 1;
    return (int)(want < cap ? want : cap);
}

hipError_t launch_prep(const ProbDev &P, hipStream_t s, const float *init_dev)
{
    if (P.prec) hipLaunchKernelGGL(k_prep, dim3(cap_grid((P.n + 255) / 256, 4096)), dim3(256), 0, s, P);
    hipLaunchKernelGGL(k_centroids<true>, dim3(cap_grid((P.kg + 3) / 4, 4096)), dim3(256), 0, s, P, init_dev);
    hipLaunchKernelGGL(k_drift, dim3(1), dim3(1024), 0, s, P, 1);
    return hipGetLastError();
}

template <bool DENSE>
static void launch_assign(const ProbDev &P, hipStream_t s, const LaunchCfg &cfg)
{
    const int threads = 64 * cfg.waves;
    const long long work = DENSE ? (P.n + 63) / 64 : (P.n + 63) / 64;
    const int grid = cap_grid((work + cfg.waves - 1) / cfg.waves, cfg.grid_cap);
    if (P.prec == 0) {
        const int dm = P.ldc;
        if (dm <= 8) hipLaunchKernelGGL((k_assign_f32<8, DENSE>), dim3(grid), dim3(threads), 0, s, P);
        else if (dm <= 16) hipLaunchKernelGGL((k_assign_f32<16, DENSE>), dim3(grid), dim3(threads), 0, s, P);
        else if (dm <= 32) hipLaunchKernelGGL((k_assign_f32<32, DENSE>), dim3(grid), dim3(threads), 0, s, P);
        else if (dm <= 64) hipLaunchKernelGGL((k_assign_f32<64, DENSE>), dim3(grid), dim3(threads), 0, s, P);
        else hipLaunchKernelGGL((k_assign_f32<128, DENSE>), dim3(grid), dim3(threads), 0, s, P);
    } else {
        switch (P.ldb / 32) {
        case 1: hipLaunchKernelGGL((k_assign_bf16<1, DENSE>), dim3(grid), dim3(threads), 0, s, P); break;
        case 2: hipLaunchKernelGGL((k_assign_bf16<2, DENSE>), dim3(grid), dim3(threads), 0, s, P); break;
        case 3: hipLaunchKernelGGL((k_assign_bf16<3, DENSE>), dim3(grid), dim3(threads), 0, s, P); break;
        case 4: hipLaunchKernelGGL((k_assign_bf16<4, DENSE>), dim3(grid), dim3(threads), 0, s, P); break;
        case 5: hipLaunchKernelGGL((k_assign_bf16<5, DENSE>), dim3(grid), dim3(threads), 0, s, P); break;
        case 6: hipLaunchKernelGGL((k_assign_bf16<6, DENSE>), dim3(grid), dim3(threads), 0, s, P); break;
        case 7: hipLaunchKernelGGL((k_assign_bf16<7, DENSE>), dim3(grid), dim3(threads), 0, s, P); break;
        default: hipLaunchKernelGGL((k_assign_bf16<8, DENSE>), dim3(grid), dim3(threads), 0, s, P); break;
        }
    }
}

static void launch_update(const ProbDev &P, hipStream_t s, const LaunchCfg &cfg)
{
    const int ublocks = cap_grid((2 * P.n + 255) / 256, cfg.grid_cap);
    hipLaunchKernelGGL(k_hist, dim3(ublocks), dim3(256), 0, s, P);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, P);
    const int sblocks = cap_grid((2 * P.n + 4095) / 4096, 1024);
    hipLaunchKernelGGL(k_scatter, dim3(sblocks), dim3(256), 0, s, P);
    const int segblocks = cap_grid((2 * P.n + 255) / 256, cfg.grid_cap);
    const int dch = (P.d + 63) / 64;
    switch (dch) {
    case 1: hipLaunchKernelGGL(k_segsum<1>, dim3(segblocks), dim3(256), 0, s, P); break;
    case 2: hipLaunchKernelGGL(k_segsum<2>, dim3(segblocks), dim3(256), 0, s, P); break;
    case 3: hipLaunchKernelGGL(k_segsum<3>, dim3(segblocks), dim3(256), 0, s, P); break;
    case 4: hipLaunchKernelGGL(k_segsum<4>, dim3(segblocks), dim3(256), 0, s, P); break;
    case 5: case 6: case 7: case 8:
        hipLaunchKernelGGL(k_segsum<8>, dim3(segblocks), dim3(256), 0, s, P); break;
    default: hipLaunchKernelGGL(k_segsum<16>, dim3(segblocks), dim3(256), 0, s, P); break;
    }
}

static void launch_centroid_rows(const ProbDev &P, hipStream_t s)
{
    hipLaunchKernelGGL(k_centroids<false>, dim3(cap_grid((P.kg + 3) / 4, 4096)), dim3(256), 0, s, P,
                       (const float *)nullptr);
    hipLaunchKernelGGL(k_drift, dim3(1), dim3(1024), 0, s, P, 0);
}

const char *stage_name(Stage st)
{
    static const char *names[ST_COUNT] = {"begin", "bound_filter", "assign_dense", "assign", "recheck",
                                          "update", "centroids"};
    return (st >= 0 && st < ST_COUNT) ? names[st] : "?";
}

int iteration_stages(const ProbDev &P, bool dense, Stage out[ST_COUNT])
{
    int n = 0;
    out[n++] = ST_BEGIN;
    if (dense) {
        out[n++] = ST_ASSIGN_DENSE;
    } else {
        out[n++] = ST_FILTER;
        out[n++] = ST_ASSIGN;
    }
    if (P.prec) out[n++] = ST_RECHECK;
    out[n++] = ST_UPDATE;
    out[n++] = ST_CENTROIDS;
    return n;
}

hipError_t launch_stage(const ProbDev &P, hipStream_t s, Stage st, bool dense, const LaunchCfg &cfg)
{
    switch (st) {
    case ST_BEGIN:
        hipLaunchKernelGGL(k_begin, dim3(cap_grid((P.kg + 256) / 256, 64)), dim3(256), 0, s, P, dense ? 1 : 0);
        break;
    case ST_FILTER:
        hipLaunchKernelGGL(k_bound_filter, dim3(cap_grid((P.n + 255) / 256, cfg.grid_cap)), dim3(256), 0, s, P);
        break;
    case ST_ASSIGN_DENSE: launch_assign<true>(P, s, cfg); break;
    case ST_ASSIGN: launch_assign<false>(P, s, cfg); break;
    case ST_RECHECK:
        hipLaunchKernelGGL(k_recheck, dim3(cap_grid((P.n + 3) / 4, cfg.grid_cap)), dim3(256), 0, s, P);
        break;
    case ST_UPDATE: launch_update(P, s, cfg); break;
    case ST_CENTROIDS: launch_centroid_rows(P, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_iteration(const ProbDev &P, hipStream_t s, bool dense, const LaunchCfg &cfg)
{
    Stage sts[ST_COUNT];
    const int n = iteration_stages(P, dense, sts);
    for (int i = 0; i < n; ++i) {
        hipError_t e = launch_stage(P, s, sts[i], dense, cfg);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_labels(const ProbDev &P, hipStream_t s, int *out)
{
    hipLaunchKernelGGL(k_labels, dim3(cap_grid((P.n + 255) / 256, 4096)), dim3(256), 0, s, P, out);
    return hipGetLastError();
}

hipError_t launch_centroids_out(const ProbDev &P, hipStream_t s, float *c32, double *c64)
{
    hipLaunchKernelGGL(k_centroids_out, dim3(cap_grid(((long long)P.kg * P.d + 255) / 256, 4096)), dim3(256), 0,
                       s, P, c32, c64);
    return hipGetLastError();
}

}  // namespace kp
