// HIP kernels (gfx950) of the filtered K-means iteration.
//
// One iteration t >= 2 of a problem runs, in stream order:
//   k_begin         clear the iteration's counters and histograms
//   k_bound_filter  point-level filter: each point's upper bound and
//                   point-level lower bound brought to this iteration; the
//                   points where ub < lbp fails form list L1  [point-level filter]
//   k_key_hist, k_scan, k_l1_scatter
//                   L1 sorted by assigned centroid (then by a bucket of the
//                   nearest other group), so that a 64-point tile shares its
//                   surviving groups
//   k_gfilter / k_group_test
//                   every group's lower bound of each point of L1 tested
//                   against its ub brought forward (its own group always
//                   open); per tile of 64 points, the list of open groups
//                                                     [group-level filter]
//   k_blk64 / k_tile_f32
//                   distances of the surviving (point, group) pairs (BF16x3
//                   on the matrix cores, or FP32 direct form); new
//                   assignment and bounds              [distance calculator]
//   k_recheck       (BF16 mode) re-decide in FP32 direct form the points whose
//                   BF16 decision is not certain under the error bound
//   k_hist, k_scan, k_scatter, k_segsum
//                   sort the moved points by centroid and add / subtract
//                   their coordinates into FP64 centroid sums    [centroid update]
//   k_centroids     new means (FP64), their FP32 / BF16 copies, drifts
//   k_drift         per-group and global maximum drift, cumulative sums
// Iteration 1 replaces the filters, the sort and the survivor form of the
// distance kernels by their dense form (every distance).  The two filters and the
// distance calculator are the three parts the paper names (Section 1); the
// result is that of standard K-means (Abstract).
#include "kp_device.h"
#include "kp_launch.h"
#include <algorithm>
#include <cmath>
#include <climits>
#include <mutex>

namespace kp {

#define KP_INF __builtin_huge_valf()

// Indices read back from memory are clamped to their arrays, so that a
// corrupted entry can only give a wrong result, never an access out of bounds.
__device__ __forceinline__ int clamp_slot(const ProbDev &P, int s) { return min(max(s, 0), P.kg - 1); }
__device__ __forceinline__ int clamp_pid(const ProbDev &P, int i) { return min(max(i, 0), (int)P.n - 1); }
// Positions of the running iteration: every point in the dense iteration,
// every entry of the sorted L1 otherwise.  Each position writes its own
// moved entry (new slot or -1) and its recheck flag, so no list is appended.
__device__ __forceinline__ long long positions(const ProbDev &P);
// A list length kept in a counter (at most one entry per point).
__device__ __forceinline__ long long list_len(const ProbDev &P, int c)
{
    const unsigned long long v = P.ctr[c];
    return v < (unsigned long long)P.n ? (long long)v : (long long)P.n;
}
__device__ __forceinline__ long long positions(const ProbDev &P)
{
    return P.ctr[CTR_DENSE] ? P.n : list_len(P, CTR_L1);
}

// =============================================================== batches
// A batched launch covers every problem of a ctx: problem i owns blocks
// tab[i] .. tab[i+1]-1 (possibly none) and runs the single-problem body with
// its own block index and count.  Returns the problem of this block.
__device__ __forceinline__ int batch_problem(const int *__restrict__ tab, int count)
{
    const int b = (int)blockIdx.x;
    int lo = 0, hi = count;   // tab[lo] <= b < tab[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tab[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

// ===================================================================== prep
// ||x||^2 of every point (FP64 sum of the FP32 coordinates' squares -- exact
// products -- in a fixed order, rounded to FP32), and their maximum
// (lbsc[2], zero before; the FP32 bits of non-negative values order as
// integers).  Sixteen lanes per point: lane l sums coordinates 4l + 64j ..
// +3 (float4 loads, so that a wave reads four rows in full lines), then a
// four-step tree within the sixteen.
__device__ __forceinline__ void b_prep(const ProbDev &P, const int bid_, const int nblk_)
{
    const int sub = lane_id() & 15;
    const int per_blk = blockDim.x / 16;
    const int64_t stride = (int64_t)nblk_ * per_blk;
    const bool vec = (P.d & 3) == 0 && ((uintptr_t)P.X & 15) == 0;
    float mx = 0.f;
    // the sixteen lanes of a point take the same trips (their shuffles stay inside the sixteen)
    for (int64_t i = (int64_t)bid_ * per_blk + threadIdx.x / 16; i < P.n; i += stride) {
        const float *x = P.X + i * P.d;
        double s = 0.0;
        if (vec) {
            for (int j = 4 * sub; j < P.d; j += 64) {
                const float4 v = *(const float4 *)(x + j);
                s += (double)v.x * v.x;
                s += (double)v.y * v.y;
                s += (double)v.z * v.z;
                s += (double)v.w * v.w;
            }
        } else {
            for (int j = sub; j < P.d; j += 16) s += (double)x[j] * x[j];
        }
        s += __shfl_xor(s, 8);
        s += __shfl_xor(s, 4);
        s += __shfl_xor(s, 2);
        s += __shfl_xor(s, 1);
        if (sub == 0) P.xn[i] = (float)s;
        mx = fmaxf(mx, (float)s);
    }
    for (int o = 32; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    if (lane_id() == 0 && mx > 0.f) atomicMax((unsigned *)&P.lbsc[2], __float_as_uint(mx));
}
__global__ __launch_bounds__(256) void k_prep(ProbDev P)
{
    b_prep(P, (int)blockIdx.x, (int)gridDim.x);
}


// ============================================================ centroid rows
// One wave per slot.  INIT: take the caller's initial centroids (original
// order).  Otherwise: c64 = sums / count (a centroid with no point keeps its
// value), then the FP32 copy, ||c32||^2 and the drift ||c32_new - c32_old||
// (FP64, rounded up).  BF16 mode: the slot's row of the matrix-core operand
// is the BF16 split of c32 for the first slot f of its 16-slot chunk and of
// c~ = fl(c32 - c32_f) for the others (the chunk's rows relative to its first
// one), with ||c~|| rounded up in nrel.  c32_f is recomputed here from the
// same sums (the wave of slot f writes the same values).
__device__ __forceinline__ double new_c64(const ProbDev &P, int s, int j, int cntv, bool init, const float *init_c)
{
    if (init) return (double)init_c[(size_t)P.perm[s] * P.d + j];
    return cntv > 0 ? P.sums[(size_t)s * P.d + j] / (double)cntv : P.c64[(size_t)s * P.d + j];
}
template <bool INIT>
__device__ __forceinline__ void b_centroids(const ProbDev &P, const int bid_, const int nblk_, const float *init)
{
    const int lane = lane_id();
    const int nw = (int)(nblk_ * blockDim.x / WAVE);
    const int L = P.prec ? P.ldb : P.ldc;
    for (int s = (int)((bid_ * blockDim.x + threadIdx.x) / WAVE); s < P.kg; s += nw) {
        const int orig = P.perm[s];
        if (orig < 0) {
            if (INIT) {
                for (int j = lane; j < L; j += WAVE) {
                    if (j < P.ldc) P.c32[(size_t)s * P.ldc + j] = 0.f;
                    if (P.prec) {
                        P.cb[(size_t)s * P.ldb + j] = 0;
                        P.cbl[(size_t)s * P.ldb + j] = 0;
                    }
                    if (j < P.d) P.c64[(size_t)s * P.d + j] = 0.0;
                }
                if (lane == 0) {
                    P.cn[s] = KP_INF;
                    P.delta[s] = 0.0;
                    P.nrel[s] = 0.f;
                }
            }
            continue;
        }
        const int cntv = INIT ? 0 : P.cnt[s];
        const int f = s & ~(CHUNK - 1);   // first slot of the chunk (always a member)
        const int cntf = INIT ? 0 : P.cnt[f];
        double dd = 0.0, q = 0.0, qr = 0.0;
        for (int j = lane; j < L; j += WAVE) {
            double c64v = 0.0, c64f = 0.0;
            float oldc = 0.f;
            if (j < P.d) {
                if (!INIT) oldc = P.c32[(size_t)s * P.ldc + j];
                c64v = new_c64(P, s, j, cntv, INIT, init);
                c64f = f == s ? c64v : new_c64(P, f, j, cntf, INIT, init);
                P.c64[(size_t)s * P.d + j] = c64v;
            }
            const float c32v = (float)c64v;
            if (j < P.ldc) P.c32[(size_t)s * P.ldc + j] = c32v;
            if (P.prec) {
                const float rel = f == s ? c32v : c32v - (float)c64f;
                const uint16_t h = f2bf(rel);
                P.cb[(size_t)s * P.ldb + j] = h;
                P.cbl[(size_t)s * P.ldb + j] = f2bf(rel - bf2f(h));
                if (f != s) qr += (double)rel * rel;
            }
            const double df = (double)c32v - (double)oldc;
            dd += df * df;
            q += (double)c32v * c32v;
        }
        dd = wave_sum_d(dd);
        q = wave_sum_d(q);
        qr = wave_sum_d(qr);
        if (lane == 0) {
            P.delta[s] = INIT ? 0.0 : sqrt(dd) * (1.0 + 0x1p-46);
            P.cn[s] = (float)q;
            if (P.prec) P.nrel[s] = qr > 0.0 ? d2f_up(sqrt(qr) * (1.0 + 0x1p-46)) : 0.f;
        }
    }
}
template <bool INIT>
__global__ __launch_bounds__(256) void k_centroids(ProbDev P, const float *init)
{
    b_centroids<INIT>(P, (int)blockIdx.x, (int)gridDim.x, init);
}
template <bool INIT>
__global__ __launch_bounds__(256) void kb_centroids(const ProbDev *__restrict__ probs, const int *__restrict__ tab, int count, const float *init)
{
    const int pi = batch_problem(tab, count);
    const ProbDev P = probs[pi];
    b_centroids<INIT>(P, (int)blockIdx.x - tab[pi], tab[pi + 1] - tab[pi], init);
}


// ================================================================== drifts
// Single workgroup.  After the update of iteration t: per-group maximum
// drift, the global maximum, the cumulative sums (FP64, each increment
// rounded up) and their FP32 copies, the groups' norm bounds and the
// iteration's statistics.  first = 1 at init.
__device__ __forceinline__ void b_drift(const ProbDev &P, const int bid_, const int nblk_, int first)
{
    __shared__ double red[1024];
    const int tid = threadIdx.x;
    const double up = 1.0 + 0x1p-50;
    double gmax = 0.0;
    if (P.prec)
        for (int ch = tid; ch < P.nch; ch += blockDim.x) {
            // (W, c W^2) of the estimate without an anchor, W >= ||c_f||
            // (cn: FP64 squared norm rounded to FP32)
            const int f = ch * CHUNK;
            P.Wu[ch] = mfma_eta3_w(d2f_up(sqrt((double)P.cn[f]) * (1.0 + 0x1p-22)));
        }
    for (int g = tid; g < P.g; g += blockDim.x) {
        double m = 0.0;
        const int s0 = P.gstart[g], ns = P.gsize[g];
        for (int r = 0; r < ns; ++r) m = fmax(m, P.delta[s0 + r]);
        // per member: how much less than the group's largest drift it moved
        for (int r = 0; r < ns; ++r) P.slk[s0 + r] = first ? 0.f : d2f_dn(fmax(m - P.delta[s0 + r], 0.0));
        const double sg = first ? 0.0 : (P.Sg[g] + m) * up;
        P.Sg[g] = sg;
        P.Sgu[g] = d2f_up(sg);
        P.Sgd[g] = d2f_dn(sg);
        gmax = fmax(gmax, m);
    }
    for (int s = tid; s < P.kg; s += blockDim.x) {
        const double sc = first ? 0.0 : (P.Sc[s] + P.delta[s]) * up;
        P.Sc[s] = sc;
        P.Scu[s] = d2f_up(sc);
        P.Scd[s] = d2f_dn(sc);
    }
    red[tid] = gmax;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (tid < o) red[tid] = fmax(red[tid], red[tid + o]);
        __syncthreads();
    }
    if (tid == 0) {
        if (first && P.prec) {
            // scale of the FP16 bound codes: a distance is at most
            // R = max ||x|| + max ||c0||; R lands in [2^10, 2^11)
            double cm = 0.0;
            for (int s = 0; s < P.kg; ++s)
                if (P.perm[s] >= 0) cm = fmax(cm, (double)P.cn[s]);
            const double R = sqrt((double)P.lbsc[2]) + sqrt(cm);
            int e = R > 0.0 ? ilogb(R) - 10 : 0;
            e = max(-100, min(100, e));
            P.lbsc[0] = ldexpf(1.f, e);
            P.lbsc[1] = ldexpf(1.f, -e);
        }
        const double sd = first ? 0.0 : (P.Sd[0] + red[0]) * up;
        P.Sd[0] = sd;
        P.Sdud[0] = d2f_up(sd);
        P.Sdud[1] = d2f_dn(sd);
        if (!first) {
            const int t = *P.iter + 1;
            long long *rec = P.stats + (size_t)((t - 1) % STATS_CAP) * 16;
            rec[0] = t;
            rec[1] = (long long)P.ctr[CTR_DENSE];
            rec[2] = list_len(P, CTR_L1);
            rec[3] = (long long)P.ctr[CTR_PAIRS];
            rec[4] = (long long)P.ctr[CTR_DIST];
            rec[5] = (long long)P.ctr[CTR_L3];
            rec[6] = (long long)P.ctr[CTR_MOVED];
            rec[7] = __double_as_longlong(red[0]);
            rec[8] = (long long)P.ctr[CTR_VISITS];
            rec[9] = (long long)P.ctr[CTR_CLOSED];
            rec[10] = *P.rowt;
            *P.iter = t;
        }
        // the next iteration tests whole bound rows in the point-level filter
        // when this one found at least an eighth of the points with every
        // group closed (the rows' extra read then costs less than the later
        // stages save on those points)
        *P.rowt = (!first && P.g <= GMAX_BF16 && 8ull * P.ctr[CTR_CLOSED] >= (unsigned long long)P.n) ? 1 : 0;
    }
}
__global__ __launch_bounds__(1024) void k_drift(ProbDev P, int first)
{
    b_drift(P, (int)blockIdx.x, (int)gridDim.x, first);
}
__global__ __launch_bounds__(1024) void kb_drift(const ProbDev *__restrict__ probs, const int *__restrict__ tab, int count, int first)
{
    const int pi = batch_problem(tab, count);
    const ProbDev P = probs[pi];
    b_drift(P, (int)blockIdx.x - tab[pi], tab[pi + 1] - tab[pi], first);
}


// ============================================================ anchor tables
// After each update (BF16 mode with anchors): Qt[a][j] = ||c32_j - c32_a||^2,
// FP64 direct form (the differences of FP32 values are exact in FP64) rounded
// to nearest FP32, +inf for a padding column; and for each chunk-first column
// j = f, Wa[a][f / 16] = (W, c W^2) with W = ||c32_f - c32_a|| (rounded up).
// One workgroup per 64 x 64 block of slot pairs with block row <= block
// column; the symmetric entries are the same sums in the same order.
constexpr int AT_T = 64;
__device__ __forceinline__ void b_atab(const ProbDev &P, int bi, int bj)
{
    __shared__ float ra[AT_T][AT_T + 1], rj[AT_T][AT_T + 1];
    if (bi > bj) return;   // uniform per workgroup
    const int t = threadIdx.x, ta = t / 16, tj = t % 16;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int c0 = 0; c0 < P.ldc; c0 += AT_T) {
        __syncthreads();
        for (int e = t; e < AT_T * AT_T; e += 256) {
            const int r = e / AT_T, c = e % AT_T;
            const int sa = bi * AT_T + r, sj = bj * AT_T + r, col = c0 + c;
            ra[r][c] = (sa < P.kg && col < P.ldc) ? P.c32[(size_t)sa * P.ldc + col] : 0.f;
            rj[r][c] = (sj < P.kg && col < P.ldc) ? P.c32[(size_t)sj * P.ldc + col] : 0.f;
        }
        __syncthreads();
        const int cn = min(AT_T, P.ldc - c0);
        for (int c = 0; c < cn; ++c) {
            double xa[4], xj[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                xa[i] = (double)ra[ta + 16 * i][c];
                xj[i] = (double)rj[tj + 16 * i][c];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const double df = xj[j] - xa[i];
                    acc[i][j] = fma(df, df, acc[i][j]);
                }
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int a = bi * AT_T + ta + 16 * i, c = bj * AT_T + tj + 16 * j;
            if (a >= P.kg || c >= P.kg) continue;
            const bool ra_ok = P.perm[a] >= 0, rc_ok = P.perm[c] >= 0;
            const float q = (float)acc[i][j];
            P.Qt[(size_t)a * P.kg + c] = rc_ok ? q : KP_INF;
            P.Qt[(size_t)c * P.kg + a] = ra_ok ? q : KP_INF;
            const float dist = d2f_up(sqrt(acc[i][j]) * (1.0 + 0x1p-40));
            if (ra_ok && (c & (CHUNK - 1)) == 0) P.Wa[(size_t)a * P.nch + c / CHUNK] = mfma_eta3_w(dist);
            if (rc_ok && (a & (CHUNK - 1)) == 0) P.Wa[(size_t)c * P.nch + a / CHUNK] = mfma_eta3_w(dist);
        }
}
__global__ __launch_bounds__(256) void k_atab(ProbDev P) { b_atab(P, (int)blockIdx.y, (int)blockIdx.x); }
__global__ __launch_bounds__(256) void kb_atab(const ProbDev *__restrict__ probs, const int *__restrict__ tab, int count)
{
    const int pi = batch_problem(tab, count);
    const ProbDev P = probs[pi];
    const int T = (P.kg + AT_T - 1) / AT_T;
    const int b = (int)blockIdx.x - tab[pi];
    b_atab(P, b / T, b % T);
}


// ================================================================= begin
__device__ __forceinline__ void b_begin(const ProbDev &P, const int bid_, const int nblk_, int dense)
{
    const int tid = bid_ * blockDim.x + threadIdx.x;
    if (tid < NCTR) P.ctr[tid] = (tid == CTR_DENSE) ? (unsigned long long)dense : 0ull;
    for (int s = tid; s <= P.kg; s += nblk_ * blockDim.x) P.hist[s] = 0;
    for (int s = tid; s <= P.nk1; s += nblk_ * blockDim.x) P.hist1[s] = 0;
}
__global__ void k_begin(ProbDev P, int dense)
{
    b_begin(P, (int)blockIdx.x, (int)gridDim.x, dense);
}
__global__ void kb_begin(const ProbDev *__restrict__ probs, const int *__restrict__ tab, int count, int dense)
{
    const int pi = batch_problem(tab, count);
    const ProbDev P = probs[pi];
    b_begin(P, (int)blockIdx.x - tab[pi], tab[pi + 1] - tab[pi], dense);
}


// ========================================================== bound filter
// Point-level filter over all points, one chunk of 16 points per thread
// (256 threads = 4096 points per workgroup step).  A point is kept in L1
// unless ub < lbp after both are brought to this iteration.  Positions come
// from one atomic per workgroup step; within it, the order is that of the
// points.
//
// lbp is brought forward by the largest drift of any centroid, which late in
// a run exceeds the gap between a point's nearest and second-nearest
// centroids for nearly every point; the group filter, which brings each
// group's bound forward by that group's own drift, then finds many points
// with every group closed (their own included).  After an iteration in which
// at least an eighth of the points were such points, the next iteration's
// filter also reads the bound row of each point that fails ub < lbp and keeps
// it only if some group is open by the group filter's test.  A point dropped
// this way keeps its assignment, state and bound row, exactly as the group
// filter would have left them (the two-level test of Section 1, applied at
// the point level).
constexpr int BF_PER_THREAD = 16;
static_assert(256 * BF_PER_THREAD == BF_CHUNK, "one bound-filter step per chunk");

// Does point i fail the point-level test ub < lbp?  (Its upper bound brought
// to this iteration is not below its point-level lower bound.)  Returns the
// state's slot, group field and that upper bound for the L1 entry.
__device__ __forceinline__ bool point_fails(const ProbDev &P, int64_t i, float sdu, int &a, int &gf, float &u)
{
    const PointState s = P.st[i];
    a = clamp_slot(P, s.a);
    gf = s.ga;
    u = ub_now(s.u, P.Scu[a]);
    return !(u < lb_now(s.p, sdu));
}
// Bits of x at multiples of np (np a power of two, at most 8) moved to
// positions 0, 1, ...: one halving per factor of two.
__device__ __forceinline__ unsigned long long gather_stride(unsigned long long x, int lnp)
{
    for (int s = 0; s < lnp; ++s) {
        x &= 0x5555555555555555ull;
        x = (x | (x >> 1)) & 0x3333333333333333ull;
        x = (x | (x >> 2)) & 0x0F0F0F0F0F0F0F0Full;
        x = (x | (x >> 4)) & 0x00FF00FF00FF00FFull;
        x = (x | (x >> 8)) & 0x0000FFFF0000FFFFull;
        x = (x | (x >> 16)) & 0x00000000FFFFFFFFull;
    }
    return x;
}
// Row test of a wave's 64 consecutive points p0 .. p0 + 63 (lane l: point
// p0 + l with ub u brought to this iteration); fm: the points that failed
// ub < lbp.  Returns the points of fm with every group closed.  np (<= 8)
// lanes read one point's row side by side, 16 bytes each (8 FP16 codes or 4
// FP32 bounds), so each load instruction covers 64 / np points' segments of
// np pieces; the np loads of a segment are all issued before the first test,
// and ballots merge the lanes' results per point.  sgu: the groups'
// cumulative drifts rounded up, in LDS.  Rows are padded to whole pieces.
template <bool C16>
__device__ __forceinline__ unsigned long long row_closed64(const ProbDev &P, int64_t p0, unsigned long long fm, float u,
                                                           const float *__restrict__ sgu)
{
    constexpr int PER = C16 ? 8 : 4;   // groups per 16-byte piece
    constexpr int ESZ = C16 ? 2 : 4;
    const int lane = lane_id(), g = P.g;
    const int need = (g + PER - 1) / PER;
    const int lnp = need <= 1 ? 0 : need <= 2 ? 1 : need <= 4 ? 2 : 3;
    const int np = 1 << lnp, ppl = 64 >> lnp;   // lanes per point, points per load
    const int q = lane >> lnp, pc = lane & (np - 1);
    const unsigned long long stride = lnp == 0 ? ~0ull : lnp == 1 ? 0x5555555555555555ull
                                    : lnp == 2 ? 0x1111111111111111ull : 0x0101010101010101ull;
    const float lsc = C16 ? P.lbsc[0] : 1.f;
    const char *rows = C16 ? (const char *)P.lbh : (const char *)P.lb;
    const size_t pitch = (size_t)P.gs * ESZ;
    unsigned long long open = 0ull;   // points with some group open
    for (int g0 = 0; g0 < g && (fm & ~open) != 0ull; g0 += np * PER) {
        const int gp = g0 + pc * PER;   // this lane's first group
        const bool gin = gp < g;
        float sv[PER];
#pragma unroll
        for (int e = 0; e < PER; ++e) sv[e] = (gin && gp + e < g) ? sgu[gp + e] : 0.f;
        const unsigned long long todo = fm & ~open;
        uint4 h[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int j = b * ppl + q;
            const bool act = b < np && gin && ((todo >> (j & 63)) & 1ull);
            h[b] = act ? *(const uint4 *)(rows + (size_t)(p0 + j) * pitch + (size_t)gp * ESZ) : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            if (b >= np) break;
            const float uj = __shfl(u, (b * ppl + q) & 63);
            const unsigned w[4] = {h[b].x, h[b].y, h[b].z, h[b].w};
            bool o = false;
#pragma unroll
            for (int e = 0; e < PER; ++e) {
                const float v = C16 ? lb16_dec((unsigned short)(w[e >> 1] >> (16 * (e & 1))), lsc) : __uint_as_float(w[e & 3]);
                o = o || (gp + e < g && group_open(uj, sv[e], v));
            }
            unsigned long long m = __ballot(o);
            for (int s = 1; s < np; s <<= 1) m |= m >> s;   // bit q np: any lane of point q
            open |= gather_stride(m & stride, lnp) << (b * ppl);
        }
    }
    return fm & ~open;
}
// Add the workgroup's count of points with every group closed (each wave's
// in its lane 0) to the iteration's counter: one atomic per workgroup.  Every
// thread of the workgroup calls it.
__device__ __forceinline__ void block_add_closed(const ProbDev &P, unsigned long long mine)
{
    __shared__ unsigned long long part[8];
    const int wv = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    if (lane_id() == 0) part[wv] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < nw; ++w) t += part[w];
        if (t) atomicAdd(&P.ctr[CTR_CLOSED], t);
    }
}

// Row pre-pass (only with the row test on): one wave per 64 consecutive
// points.  Each lane tests its point's ub < lbp, the wave runs the row test
// on the points that fail it, and the mask of the points with every group
// closed is stored as two words of rclosed, which the bound filter then
// reads.  The groups' drifts are copied to LDS (g <= GMAX_BF16 whenever the
// row test is on).
__device__ __forceinline__ void b_row_pre(const ProbDev &P, const int bid_, const int nblk_)
{
    __shared__ float sgu_l[GMAX_BF16];
    if (*P.rowt == 0) return;   // uniform: the gate of this iteration
    for (int i = threadIdx.x; i < (P.g + 63) / 64 * 64; i += blockDim.x) sgu_l[i] = i < P.g ? P.Sgu[i] : 0.f;
    __syncthreads();
    const int lane = lane_id(), wv = threadIdx.x / WAVE;
    const bool c16 = P.prec && P.lb16;
    const float sdu = P.Sdud[0];
    const int64_t nw = (P.n + 63) / 64;
    unsigned long long n_closed = 0;
    for (int64_t w = (int64_t)bid_ * 4 + wv; w < nw; w += (int64_t)nblk_ * 4) {
        const int64_t p0 = w * 64, i = p0 + lane;
        int a = 0, gf = 0;
        float u = 0.f;
        const bool f = i < P.n && point_fails(P, i, sdu, a, gf, u);
        const unsigned long long fm = __ballot(f);
        const unsigned long long cm = fm == 0ull ? 0ull
                                      : (c16 ? row_closed64<true>(P, p0, fm, u, sgu_l)
                                             : row_closed64<false>(P, p0, fm, u, sgu_l));
        if (lane < 2) P.rclosed[2 * w + lane] = (unsigned)(cm >> (32 * lane));
        n_closed += (unsigned long long)__popcll(cm);
    }
    block_add_closed(P, n_closed);
}
__global__ __launch_bounds__(256) void k_row_pre(ProbDev P) { b_row_pre(P, (int)blockIdx.x, (int)gridDim.x); }
__global__ __launch_bounds__(256) void kb_row_pre(const ProbDev *__restrict__ probs, const int *__restrict__ tab, int count)
{
    const int pi = batch_problem(tab, count);
    const ProbDev P = probs[pi];
    b_row_pre(P, (int)blockIdx.x - tab[pi], tab[pi + 1] - tab[pi]);
}
// Does point i go to L1: it fails ub < lbp and, with the row test on, the
// row pre-pass found some group open.
__device__ __forceinline__ bool point_kept(const ProbDev &P, int64_t i, float sdu, bool rowt, int &a, int &gf, float &u)
{
    if (!point_fails(P, i, sdu, a, gf, u)) return false;
    return !rowt || !((P.rclosed[i >> 5] >> (i & 31)) & 1u);
}

// Deterministic mode, first pass: failures per chunk of BF_CHUNK points.
__device__ __forceinline__ void b_bf_count(const ProbDev &P, const int bid_, const int nblk_)
{
    __shared__ int wcount[4];
    const int tid = threadIdx.x, lane = lane_id(), wv = tid / WAVE;
    const float sdu = P.Sdud[0];
    const bool rowt = *P.rowt != 0;
    for (int64_t b0 = (int64_t)bid_ * BF_CHUNK; b0 < P.n; b0 += (int64_t)nblk_ * BF_CHUNK) {
        int mine = 0;
#pragma unroll 4
        for (int r = 0; r < BF_PER_THREAD; ++r) {
            const int64_t i = b0 + (int64_t)r * 256 + tid;
            int a, gf;
            float u;
            const bool keep = i < P.n && point_kept(P, i, sdu, rowt, a, gf, u);
            mine += __popcll(__ballot(keep));
        }
        if (lane == 0) wcount[wv] = mine;
        __syncthreads();
        if (tid == 0) P.dcnt[b0 / BF_CHUNK] = wcount[0] + wcount[1] + wcount[2] + wcount[3];
        __syncthreads();
    }
}
__global__ __launch_bounds__(256) void k_bf_count(ProbDev P) { b_bf_count(P, (int)blockIdx.x, (int)gridDim.x); }

__device__ __forceinline__ void b_bound_filter(const ProbDev &P, const int bid_, const int nblk_)
{
    __shared__ int wcount[4];
    __shared__ unsigned long long base_s;
    const int tid = threadIdx.x, lane = lane_id(), wv = tid / WAVE;
    const float sdu = P.Sdud[0];
    const bool rowt = *P.rowt != 0;
    const int64_t chunk = 256 * BF_PER_THREAD;
    for (int64_t b0 = (int64_t)bid_ * chunk; b0 < P.n; b0 += (int64_t)nblk_ * chunk) {
        unsigned long long masks[BF_PER_THREAD];
        int ka[BF_PER_THREAD], kgf[BF_PER_THREAD];   // the kept points' slot and group field
        float ku[BF_PER_THREAD];                     // and upper bound brought to this iteration
        int mine = 0;
#pragma unroll
        for (int r = 0; r < BF_PER_THREAD; ++r) {
            const int64_t i = b0 + (int64_t)r * 256 + tid;
            ka[r] = 0;
            kgf[r] = 0;
            ku[r] = 0.f;
            const bool keep = i < P.n && point_kept(P, i, sdu, rowt, ka[r], kgf[r], ku[r]);
            masks[r] = __ballot(keep);
            mine += __popcll(masks[r]);
        }
        if (lane == 0) wcount[wv] = mine;
        __syncthreads();
        if (tid == 0) {
            const int tot = wcount[0] + wcount[1] + wcount[2] + wcount[3];
            // deterministic mode: the chunk's place from the scan of the
            // per-chunk counts (chunk order); otherwise first come, first served
            base_s = P.det ? (unsigned long long)P.doff[b0 / BF_CHUNK]
                           : (tot ? atomicAdd(&P.ctr[CTR_L1], (unsigned long long)tot) : 0ull);
        }
        __syncthreads();
        unsigned long long pos = base_s;
        for (int w = 0; w < wv; ++w) pos += (unsigned long long)wcount[w];
        const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
        for (int r = 0; r < BF_PER_THREAD; ++r) {
            if ((masks[r] >> lane) & 1ull)
                P.L1[pos + __popcll(masks[r] & below)] =
                    make_int4((int)(b0 + (int64_t)r * 256 + tid), ka[r], __float_as_int(ku[r]), kgf[r]);
            pos += (unsigned long long)__popcll(masks[r]);
        }
        __syncthreads();
    }
}
__global__ __launch_bounds__(256) void k_bound_filter(ProbDev P)
{
    b_bound_filter(P, (int)blockIdx.x, (int)gridDim.x);
}
__global__ __launch_bounds__(256) void kb_bound_filter(const ProbDev *__restrict__ probs, const int *__restrict__ tab, int count)
{
    const int pi = batch_problem(tab, count);
    const ProbDev P = probs[pi];
    b_bound_filter(P, (int)blockIdx.x - tab[pi], tab[pi + 1] - tab[pi]);
}


// ======================================================= L1 sort by slot
// key of L1 entry e: the slot its point is assigned to.
// Key of an L1 entry: its slot, then one of nk1 / kg buckets of the nearest
// other group of its last decision (the group modulo the bucket count), so
// that a tile's points tend to share their neighbouring groups as well as
// their own.  The key space stays within the LDS histogram.
__device__ __forceinline__ int l1_key(const ProbDev &P, int a, int gaf)
{
    const int nb = P.nk1 / P.kg;
    if (nb <= 1) return a;
    const int o = min((gaf >> 16) & 0xFFFF, P.g);   // 0xFFFF (none) -> group g
    return a * nb + o % nb;
}

__device__ __forceinline__ void b_key_hist(const ProbDev &P, const int bid_, const int nblk_)
{
    __shared__ int h[L1_HIST];
    const long long n1 = list_len(P, CTR_L1);
    const bool lds = P.nk1 <= L1_HIST;
    if (lds)
        for (int i = threadIdx.x; i < P.nk1; i += blockDim.x) h[i] = 0;
    __syncthreads();
    for (long long e = (long long)bid_ * blockDim.x + threadIdx.x; e < n1;
         e += (long long)nblk_ * blockDim.x) {
        const int4 u = P.L1[e];
        const int key = l1_key(P, clamp_slot(P, u.y), u.w);
        if (lds) atomicAdd(&h[key], 1);
        else atomicAdd(&P.hist1[key], 1);
    }
    __syncthreads();
    if (lds)
        for (int i = threadIdx.x; i < P.nk1; i += blockDim.x)
            if (h[i]) atomicAdd(&P.hist1[i], h[i]);
}
__global__ __launch_bounds__(256) void k_key_hist(ProbDev P)
{
    b_key_hist(P, (int)blockIdx.x, (int)gridDim.x);
}
__global__ __launch_bounds__(256) void kb_key_hist(const ProbDev *__restrict__ probs, const int *__restrict__ tab, int count)
{
    const int pi = batch_problem(tab, count);
    const ProbDev P = probs[pi];
    b_key_hist(P, (int)blockIdx.x - tab[pi], tab[pi + 1] - tab[pi]);
}


// Exclusive scan of hist[0..n) into cursor (single workgroup of 1024).
__device__ __forceinline__ void b_scan(const int *hist, int *cursor, int n)
{
    __shared__ int part[1024];
    const int tid = threadIdx.x;
    const int per = (n + 1023) / 1024;
    const int b = tid * per, e = min(n, b + per);
    int s = 0;
    for (int i = b; i < e; ++i) s += hist[i];
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
        cursor[i] = run;
        run += hist[i];
    }
}
__global__ __launch_bounds__(1024) void k_scan(const int *hist, int *cursor, int n) { b_scan(hist, cursor, n); }
// One workgroup per problem: which = 1 scans the L1 sort histogram, 0 the update one.
__global__ __launch_bounds__(1024) void kb_scan(const ProbDev *__restrict__ probs, const int *__restrict__ tab, int count, int which)
{
    const ProbDev P = probs[batch_problem(tab, count)];
    if (which) b_scan(P.hist1, P.cursor1, P.nk1);
    else b_scan(P.hist, P.cursor, P.kg);
}


__device__ __forceinline__ void b_l1_scatter(const ProbDev &P, const int bid_, const int nblk_)
{
    __shared__ int h[L1_HIST];   // this workgroup's count per key, then its next position per key
    const long long E = list_len(P, CTR_L1);
    const long long b0 = E * bid_ / nblk_, b1 = E * (bid_ + 1) / nblk_;
    if (P.nk1 > L1_HIST) {
        for (long long e = b0 + threadIdx.x; e < b1; e += blockDim.x) {
            const int4 u = P.L1[e];
            const int pid = clamp_pid(P, u.x), a = clamp_slot(P, u.y), key = l1_key(P, a, u.w);
            const int pos = atomicAdd(&P.cursor1[key], 1);
            if (P.prec) P.L1x[pos] = make_int4(pid, a, u.z, u.w & 0xFFFF);   // BF16 mode reads only L1x
            else P.L1s[pos] = pid;
        }
        return;
    }
    if (b0 >= b1) return;   // uniform per block
    for (int i = threadIdx.x; i < P.nk1; i += blockDim.x) h[i] = 0;
    __syncthreads();
    for (long long e = b0 + threadIdx.x; e < b1; e += blockDim.x) {
        const int4 u = P.L1[e];
        atomicAdd(&h[l1_key(P, clamp_slot(P, u.y), u.w)], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < P.nk1; i += blockDim.x) h[i] = h[i] ? atomicAdd(&P.cursor1[i], h[i]) : 0;
    __syncthreads();
    for (long long e = b0 + threadIdx.x; e < b1; e += blockDim.x) {
        const int4 u = P.L1[e];
        const int pid = clamp_pid(P, u.x), a = clamp_slot(P, u.y), key = l1_key(P, a, u.w);
        const int pos = atomicAdd(&h[key], 1);
        if (P.prec) P.L1x[pos] = make_int4(pid, a, u.z, u.w & 0xFFFF);   // BF16 mode reads only L1x
        else P.L1s[pos] = pid;
    }
}
__global__ __launch_bounds__(256) void k_l1_scatter(ProbDev P)
{
    b_l1_scatter(P, (int)blockIdx.x, (int)gridDim.x);
}
__global__ __launch_bounds__(256) void kb_l1_scatter(const ProbDev *__restrict__ probs, const int *__restrict__ tab, int count)
{
    const int pi = batch_problem(tab, count);
    const ProbDev P = probs[pi];
    b_l1_scatter(P, (int)blockIdx.x - tab[pi], tab[pi + 1] - tab[pi]);
}


// ===================================================== FP32 direct distance
// Squared distance in the direct form with accumulator i mod 4 (see
// eps2_direct).  x has `DMAX` registers, zero beyond d; c is a row padded
// with zeros to ldc (a multiple of 4).
template <int DMAX>
__device__ __forceinline__ float direct_d2(const float (&x)[DMAX], const float *__restrict__ c, int ldc)
{
    // Blocks of up to 32 coordinates: every load of a block is issued before
    // the first product, so a row costs one memory latency per block.  Pieces
    // past ldc read the row's last piece (a clamped address) and are weighted
    // by 0, making their terms exact zeros.  The loaded values are used with
    // no condition: a use under a branch would let the compiler move each
    // load into its own branch and wait for it there.
    constexpr int B = DMAX < 32 ? DMAX : 32;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
#pragma unroll
    for (int i0 = 0; i0 < DMAX; i0 += B) {
        if (i0 < ldc) {
            float4 cv[B / 4];
#pragma unroll
            for (int q = 0; q < B / 4; ++q) cv[q] = *(const float4 *)(c + min(i0 + 4 * q, ldc - 4));
#pragma unroll
            for (int q = 0; q < B / 4; ++q) {
                const int i = i0 + 4 * q;
                const float w = i < ldc ? 1.f : 0.f;
                const float t0 = (x[i] - cv[q].x) * w, t1 = (x[i + 1] - cv[q].y) * w;
                const float t2 = (x[i + 2] - cv[q].z) * w, t3 = (x[i + 3] - cv[q].w) * w;
                a0 = fmaf(t0, t0, a0);
                a1 = fmaf(t1, t1, a1);
                a2 = fmaf(t2, t2, a2);
                a3 = fmaf(t3, t3, a3);
            }
        }
    }
    return (a0 + a1) + (a2 + a3);
}

// Same arithmetic with both rows read from memory (x unpadded, length d; c
// padded with zeros to a multiple of 4).
__device__ __forceinline__ float direct_d2_mem(const float *__restrict__ x, const float *__restrict__ c, int d)
{
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    if ((d & 3) == 0) {
        for (int i = 0; i < d; i += 4) {
            const float4 xv = *(const float4 *)(x + i);
            const float4 cv = *(const float4 *)(c + i);
            const float t0 = xv.x - cv.x, t1 = xv.y - cv.y, t2 = xv.z - cv.z, t3 = xv.w - cv.w;
            a0 = fmaf(t0, t0, a0);
            a1 = fmaf(t1, t1, a1);
            a2 = fmaf(t2, t2, a2);
            a3 = fmaf(t3, t3, a3);
        }
    } else {
        for (int i = 0; i < d; i += 4) {
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

// Direct form on BF16 rows (both padded with zeros to ldb): the differences
// of BF16 values are exact in FP32, so the result is ||xb - cb||^2 with the
// relative error of eps2_direct(ldb).
__device__ __forceinline__ float direct_d2_bf16(const uint16_t *__restrict__ x, const uint16_t *__restrict__ c,
                                                int ldb)
{
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    for (int i = 0; i < ldb; i += 8) {
        const uint4 xv = *(const uint4 *)(x + i);
        const uint4 cv = *(const uint4 *)(c + i);
        const unsigned xs[4] = {xv.x, xv.y, xv.z, xv.w}, cs[4] = {cv.x, cv.y, cv.z, cv.w};
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const float tlo = __uint_as_float(xs[w] << 16) - __uint_as_float(cs[w] << 16);
            const float thi = __uint_as_float(xs[w] & 0xFFFF0000u) - __uint_as_float(cs[w] & 0xFFFF0000u);
            // coordinates i + 2w (accumulator 2w mod 4) and i + 2w + 1
            if (w & 1) {
                a2 = fmaf(tlo, tlo, a2);
                a3 = fmaf(thi, thi, a3);
            } else {
                a0 = fmaf(tlo, tlo, a0);
                a1 = fmaf(thi, thi, a1);
            }
        }
    }
    return (a0 + a1) + (a2 + a3);
}

// Is (v, slot sa) before (w, slot sb) in (distance, original index) order?
// A slot outside 0..kg-1 (the "none yet" -1 or a skipped block's sentinel)
// never wins and loses every tie.
__device__ __forceinline__ bool before(const ProbDev &P, float v, int sa, float w, int sb)
{
    if ((unsigned)sa >= (unsigned)P.kg) return false;
    if (v < w) return true;
    if (v > w) return false;
    if ((unsigned)sb >= (unsigned)P.kg) return true;
    return P.perm[sa] < P.perm[sb];
}


// ====================================================== per-point decisions
// Running best of one point over the groups examined: best value, its slot
// and group, the second value of the best's group and the overall second;
// ov / og: the smallest value of any other group and that group (the point's
// nearest other group, kept for the order of the next iteration's L1).
struct Run {
    float bd, sec, bm2, ov;
    float lk;   // smallest lower bound (a distance) of the centroids the local filter skipped
    int bs, bg, og;
};
__device__ __forceinline__ void run_init(Run &r)
{
    r.lk = KP_INF;
    r.bd = KP_INF;
    r.sec = KP_INF;
    r.bm2 = KP_INF;
    r.ov = KP_INF;
    r.bs = -1;
    r.bg = -1;
    r.og = -1;
}
// The state's group field: the assigned centroid's group in the low 16 bits,
// the nearest other group (0xFFFF: none) in the high 16.
__device__ __forceinline__ int pack_ga(int ga, int og)
{
    const unsigned o = (og >= 0 && og != ga) ? (unsigned)og & 0xFFFFu : 0xFFFFu;
    return (int)(((unsigned)ga & 0xFFFFu) | (o << 16));
}
__device__ __forceinline__ void run_fold(const ProbDev &P, Run &r, const Best3 &gb, int g)
{
    // A group result of +inf carries no slot (a skipped MFMA block): never a best.
    if (!(gb.m1 < KP_INF)) return;
    if (before(P, gb.m1, gb.s1, r.bd, r.bs)) {
        if (g != r.bg) {   // the old best's group is now the nearest other one
            r.ov = r.bd;
            r.og = r.bg;
        }
        r.sec = fminf(r.bd, gb.m2);
        r.bd = gb.m1;
        r.bs = gb.s1;
        r.bg = g;
        r.bm2 = gb.m2;
    } else {
        r.sec = fminf(r.sec, gb.m1);
        if (g != r.bg && gb.m1 < r.ov) {
            r.ov = gb.m1;
            r.og = g;
        }
    }
}

// FP32 direct distances of a lane's point (x in registers) to every member of
// group g; the rows are uniform across the wave (scalar loads).
template <int DMAX>
__device__ __forceinline__ Best3 direct_group(const ProbDev &P, int g, const float (&x)[DMAX])
{
    Best3 b = {KP_INF, -1, KP_INF};
    const int s0 = P.gstart[g], ns = P.gsize[g];
    for (int r = 0; r < ns; ++r) {
        const float v = direct_d2<DMAX>(x, P.c32 + (size_t)(s0 + r) * P.ldc, P.ldc);
        if (v < b.m1) {
            b.m2 = b.m1;
            b.m1 = v;
            b.s1 = s0 + r;
        } else {
            b.m2 = fminf(b.m2, v);
        }
    }
    return b;
}

// FP32 decision and writes (no recheck: decisions on direct FP32 values).
// `r` already holds the old centroid when a_sep.
__device__ __forceinline__ bool finish_f32(const ProbDev &P, int pid, bool dense, int a, int ga, bool a_sep,
                                           float d2a, float lbe_a, float minnc, const Run &r, double eps2,
                                           float sdd)
{
    float *lbrow = P.lb + (size_t)pid * P.gs;
    if (r.bg >= 0) lbrow[r.bg] = store_lb(dist_lo(r.bm2, eps2), P.Sgd[r.bg]);
    float lbp = fminf(fminf(dist_lo(r.sec, eps2), minnc), r.lk);
    if (!dense && a_sep && r.bs != a) {
        const float va = fminf(lbe_a, dist_lo(d2a, eps2));
        lbrow[ga] = store_lb(va, P.Sgd[ga]);
        lbp = fminf(lbp, va);
    }
    // r.bs >= 0 whenever some distance was finite; otherwise keep the old slot
    const int win = r.bs >= 0 ? r.bs : (a >= 0 ? a : 0);
    PointState ns;
    ns.a = win;
    ns.u = store_u(dist_hi(r.bd, eps2), P.Scd[win]);
    ns.p = store_lb(lbp, sdd);
    ns.ga = pack_ga(P.slot_group[win], win == r.bs ? r.og : -1);
    P.st[pid] = ns;
    return win != (dense ? -1 : a);
}

// ============================================== BF16 engine: MFMA per group
// A FP32 vector is split as x = xh + xl + rx with xh = bf16(x) and
// xl = bf16(x - xh) (x - xh is exact in FP32); the centroids the same way
// (cb, cbl).  The dot product x.c is taken as xh.ch + (xl.ch + xh.cl),
// accumulated on the matrix cores (v_mfma_f32_16x16x32_bf16: exact products,
// FP32 sums) in two accumulators, one for the leading products and one for
// the two correction products; mfma_eta3 bounds the error of the resulting
// squared distance.
//
// One wave works on a tile of 16 points.  Lane l holds point (l & 15) of the
// tile and coordinates 32 ks + 8 (l >> 4) .. +7 of its split row: the B
// operand.  With A = a 16-slot chunk of one group (rows slot0 + (l & 15)),
// the product gives lane l the estimates of its point against slots
// slot0 + 4 (l >> 4) .. +3.
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

template <int KS>
struct PtFrag {
    bf16x8 h[KS], l[KS];
};

// Split of 8 FP32 values (conversions round to nearest even).
__device__ __forceinline__ void split8(const float (&v)[8], bf16x8 &h, bf16x8 &l)
{
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const __bf16 t = (__bf16)v[j];
        h[j] = t;
        l[j] = (__bf16)(v[j] - (float)t);
    }
}

// The tile's B operand from the FP32 rows; zero beyond d and for absent
// points.  With crow (OWN): also this lane's part of the FP32 direct-form
// squared distance to that centroid row (c32, padded with zeros to ldc):
// the lane's 8 KS coordinates summed in order with fused multiply-adds; the
// four lanes of a point are combined by the caller (eps2_tile bounds it).
// This lane's 8 KS coordinates of point pid (FP32, zero beyond d and for
// absent points): coordinates 32 ks + 8 (l >> 4) .. +7 for ks < KS.
template <int KS>
__device__ __forceinline__ void load_rows16(const ProbDev &P, int pid, bool ok, float (&v)[KS][8])
{
    const int quad = lane_id() >> 4;
    const float *xr = P.X + (size_t)pid * P.d;
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    if ((P.d & 3) == 0 && ((uintptr_t)P.X & 15) == 0) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int k0 = 32 * ks + 8 * quad;   // d % 4 == 0: a float4 is wholly inside or outside
            const float4 p0 = (ok && k0 < P.d) ? *(const float4 *)(xr + k0) : z;
            const float4 p1 = (ok && k0 + 4 < P.d) ? *(const float4 *)(xr + k0 + 4) : z;
            v[ks][0] = p0.x;
            v[ks][1] = p0.y;
            v[ks][2] = p0.z;
            v[ks][3] = p0.w;
            v[ks][4] = p1.x;
            v[ks][5] = p1.y;
            v[ks][6] = p1.z;
            v[ks][7] = p1.w;
        }
    } else {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = 32 * ks + 8 * quad + j;
                v[ks][j] = (ok && k < P.d) ? xr[k] : 0.f;
            }
    }
}

// The tile's B operand from the FP32 rows; zero beyond d and for absent
// points.  With crow (OWN): also this lane's part of the FP32 direct-form
// squared distance to that centroid row (c32, padded with zeros to ldc):
// the lane's 8 KS coordinates summed in order with fused multiply-adds; the
// four lanes of a point are combined by the caller (eps2_tile bounds it).
template <int KS, bool OWN>
__device__ __forceinline__ float load_points16(const ProbDev &P, int pid, bool ok, const float *crow, PtFrag<KS> &b)
{
    const int quad = lane_id() >> 4;
    float v[KS][8], c[KS][8];
    load_rows16<KS>(P, pid, ok, v);
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    float d2 = 0.f;
    if (OWN) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int k0 = 32 * ks + 8 * quad;   // ldc % 4 == 0 and the row is 16-byte aligned
            const float4 q0 = (ok && k0 < P.ldc) ? *(const float4 *)(crow + k0) : z;
            const float4 q1 = (ok && k0 + 4 < P.ldc) ? *(const float4 *)(crow + k0 + 4) : z;
            c[ks][0] = q0.x;
            c[ks][1] = q0.y;
            c[ks][2] = q0.z;
            c[ks][3] = q0.w;
            c[ks][4] = q1.x;
            c[ks][5] = q1.y;
            c[ks][6] = q1.z;
            c[ks][7] = q1.w;
        }
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const float t = v[ks][j] - c[ks][j];
                d2 = fmaf(t, t, d2);
            }
    }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) split8(v[ks], b.h[ks], b.l[ks]);
    return d2;
}
// Relative error of that distance after combining the four lanes: each of
// the 8 KS terms adds one rounding to its lane's sum, each rounded
// difference squared 2u, the two combining adds 2u; doubled as margin.
__host__ __device__ __forceinline__ double eps2_tile(int ks)
{
    return (double)(8 * ks + 8) * 2.0 * 5.9604644775390625e-08;
}

// Per-point results of a chunk in key form.  Each row j of the chunk gives a
// squared lower bound L_j = fl(v_j - e_j) and upper bound U_j = fl(v_j + e_j)
// of ||x - c_j||^2 (see the bound of the estimates).  A key is L_j's FP32
// bits with the low 4 bits cleared (so at most 2^-19 relative below L_j:
// still a lower bound) and the row's offset in the chunk in those 4 bits;
// unsigned order of keys is the order of the truncated bounds, ties to the
// lower slot.  k1 <= k2 are the two smallest keys and u1 the upper bound of
// k1's row.
struct Key3 {
    unsigned k1, k2;
    float u1;
};
__device__ __forceinline__ Key3 key3_empty() { return Key3{0xFFFFFFFFu, 0xFFFFFFFFu, KP_INF}; }
__device__ __forceinline__ Key3 key3_merge(Key3 a, Key3 b)
{
    const bool ta = a.k1 < b.k1;
    Key3 r;
    r.k1 = ta ? a.k1 : b.k1;
    r.u1 = ta ? a.u1 : b.u1;
    r.k2 = min(ta ? b.k1 : a.k1, min(a.k2, b.k2));
    return r;
}
// v_permlane16_swap(X, Y) swaps the odd 16-lane rows of X with the even rows
// of Y: afterwards X = [X0, Y0, X2, Y2] and Y = [X1, Y1, X3, Y3] by rows.
// v_permlane32_swap(X, Y) swaps the upper half of X with the lower half of
// Y: X = [X0, X1, Y0, Y1], Y = [X2, X3, Y2, Y3].  With X = Y every lane gets
// its own value and its partner's (l ^ 16, l ^ 32); the symmetric merge
// takes them in a fixed order, so both partners agree.  All 64 lanes must be
// active.
__device__ __forceinline__ Key3 key3_swap16(Key3 x, Key3 y, bool first)
{
    const auto a = __builtin_amdgcn_permlane16_swap(x.k1, y.k1, false, false);
    const auto b = __builtin_amdgcn_permlane16_swap(x.k2, y.k2, false, false);
    const auto c = __builtin_amdgcn_permlane16_swap(__float_as_uint(x.u1), __float_as_uint(y.u1), false, false);
    return first ? Key3{a[0], b[0], __uint_as_float(c[0])} : Key3{a[1], b[1], __uint_as_float(c[1])};
}
__device__ __forceinline__ void key3_swap16_both(Key3 x, Key3 y, Key3 &nx, Key3 &ny)
{
    const auto a = __builtin_amdgcn_permlane16_swap(x.k1, y.k1, false, false);
    const auto b = __builtin_amdgcn_permlane16_swap(x.k2, y.k2, false, false);
    const auto c = __builtin_amdgcn_permlane16_swap(__float_as_uint(x.u1), __float_as_uint(y.u1), false, false);
    nx = Key3{a[0], b[0], __uint_as_float(c[0])};
    ny = Key3{a[1], b[1], __uint_as_float(c[1])};
}
__device__ __forceinline__ void key3_swap32_both(Key3 x, Key3 y, Key3 &nx, Key3 &ny)
{
    const auto a = __builtin_amdgcn_permlane32_swap(x.k1, y.k1, false, false);
    const auto b = __builtin_amdgcn_permlane32_swap(x.k2, y.k2, false, false);
    const auto c = __builtin_amdgcn_permlane32_swap(__float_as_uint(x.u1), __float_as_uint(y.u1), false, false);
    nx = Key3{a[0], b[0], __uint_as_float(c[0])};
    ny = Key3{a[1], b[1], __uint_as_float(c[1])};
}
// The lane's partial (its four rows) merged over the four rows of lanes:
// every lane of point p returns the chunk's result for p.
__device__ __forceinline__ Key3 key3_fold_all(Key3 t)
{
    Key3 x, y;
    key3_swap16_both(t, t, x, y);
    t = key3_merge(x, y);
    key3_swap32_both(t, t, x, y);
    return key3_merge(x, y);
}
// Four chunks' partials p[0..3] of this lane's point reduced and spread:
// the lane in row q returns chunk q's result for its point.  The first swap
// leaves in even rows chunk 0 (2) merged over the row pair, in odd rows
// chunk 1 (3); the second pairs rows 0/2 and 1/3.
__device__ __forceinline__ Key3 key3_scatter4(const Key3 &p0, const Key3 &p1, const Key3 &p2, const Key3 &p3)
{
    Key3 a, b, c, d;
    key3_swap16_both(p0, p1, a, b);
    const Key3 q01 = key3_merge(a, b);
    key3_swap16_both(p2, p3, c, d);
    const Key3 q23 = key3_merge(c, d);
    key3_swap32_both(q01, q23, a, b);
    return key3_merge(a, b);
}
__device__ __forceinline__ float key_value(unsigned k) { return __uint_as_float(k & ~15u); }

// Bounds on the true distance from bounds of its square: v_sqrt_f32 is
// within 1 ulp of the square root (normal inputs); two steps cover it.  Tiny
// arguments give the lower bound 0.
__device__ __forceinline__ float sq_lo(float v, float eta_f) { return dn_nonneg(v - eta_f); }
__device__ __forceinline__ float root_lo(float t)
{
    return t > 0x1p-100f ? __uint_as_float(__float_as_uint(__builtin_amdgcn_sqrtf(t)) - 2u) : 0.f;
}
__device__ __forceinline__ float root_hi(float t)
{
    if (!(t < __builtin_huge_valf())) return t;
    return __uint_as_float(__float_as_uint(__builtin_amdgcn_sqrtf(fmaxf(t, 0x1p-100f))) + 2u);
}

// Running best of a point over chunk results: the best is the row with the
// smallest squared lower bound bdl (slot bs in group bg, squared upper bound
// bu); every other row enters by its squared lower bound (root_lo is
// monotone, so minima carry over): sec over all of them, bm2 over the best's
// group, ov (nearest other group, for the L1 order only) over the other
// groups.
struct RunB {
    float bdl, bu, sec, bm2, ov;
    int bs, bg, og;
    int wq;   // the row of lanes that folded the best (it stored the best group's bound)
};
__device__ __forceinline__ void runb_init(RunB &r)
{
    r.wq = 0;
    r.bdl = KP_INF;
    r.bu = KP_INF;
    r.sec = KP_INF;
    r.bm2 = KP_INF;
    r.ov = KP_INF;
    r.bs = -1;
    r.bg = -1;
    r.og = -1;
}
// Fold one chunk of group g, when `on`: smallest lower bound l1 at slot s1
// with upper bound u1, the second smallest l2, and gprev the smallest lower
// bound of the group's earlier chunks (+inf for its first).  Equal bounds can
// never be decided, so ties keep the earlier result.
__device__ __forceinline__ void runb_fold(RunB &r, bool on, float l1, float u1, int s1, float l2, int g, float gprev,
                                          bool track_og)
{
    const bool nb = on && l1 < r.bdl;
    // the old best (and everything below it) becomes an other row
    const float sec = nb ? fminf(fminf(r.bdl, r.sec), l2) : fminf(r.sec, l1);
    const float bm2 = nb ? fminf(l2, gprev) : (g == r.bg ? fminf(r.bm2, l1) : r.bm2);
    if (track_og) {   // wave-uniform
        // nearest other group: the old best's group when a new group leads,
        // else this group when it comes closer than the current one
        const float gm = fminf(gprev, l1);
        const bool oo = nb && g != r.bg;
        const bool on2 = on && !nb && g != r.bg && gm < r.ov;
        r.ov = oo ? r.bdl : (on2 ? gm : r.ov);
        r.og = oo ? r.bg : (on2 ? g : r.og);
    }
    r.sec = on ? sec : r.sec;
    r.bm2 = on ? bm2 : r.bm2;
    r.bdl = nb ? l1 : r.bdl;
    r.bu = nb ? u1 : r.bu;
    r.bs = nb ? s1 : r.bs;
    r.bg = nb ? g : r.bg;
    r.wq = nb ? (lane_id() >> 4) : r.wq;
}
// Two running bests over disjoint sets of groups (the lanes of one point
// that handled different chunks), merged; a and b are the states of the
// lower and the upper lane of the pair, so both lanes compute the same.
__device__ __forceinline__ RunB runb_merge(const RunB &a, const RunB &b)
{
    const bool tb = b.bdl < a.bdl;
    const RunB &w = tb ? b : a, &l = tb ? a : b;
    RunB r = w;
    r.sec = fminf(fminf(w.sec, l.sec), l.bdl);
    // nearest other group: the winner's, the loser's best group or its other
    float ov = w.ov;
    int og = w.og;
    if (l.bg >= 0 && l.bdl < ov) {
        ov = l.bdl;
        og = l.bg;
    }
    if (l.og >= 0 && l.ov < ov) {
        ov = l.ov;
        og = l.og;
    }
    r.ov = ov;
    r.og = og;
    return r;
}
__device__ __forceinline__ RunB runb_swap(const RunB &x, bool half32, bool upper)
{
    auto sw = [&](unsigned v) {
        const auto t = half32 ? __builtin_amdgcn_permlane32_swap(v, v, false, false)
                              : __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return upper ? t[1] : t[0];
    };
    RunB r;
    r.bdl = __uint_as_float(sw(__float_as_uint(x.bdl)));
    r.bu = __uint_as_float(sw(__float_as_uint(x.bu)));
    r.sec = __uint_as_float(sw(__float_as_uint(x.sec)));
    r.bm2 = __uint_as_float(sw(__float_as_uint(x.bm2)));
    r.ov = __uint_as_float(sw(__float_as_uint(x.ov)));
    r.bs = (int)sw((unsigned)x.bs);
    r.bg = (int)sw((unsigned)x.bg);
    r.og = (int)sw((unsigned)x.og);
    r.wq = (int)sw((unsigned)x.wq);
    return r;
}
// The four lanes of a point (rows 0..3) hold running bests over disjoint
// chunks; afterwards each holds the merge of all four.
__device__ __forceinline__ RunB runb_allreduce(const RunB &r)
{
    const RunB e16 = runb_swap(r, false, false), o16 = runb_swap(r, false, true);   // rows (0|2) and (1|3)
    const RunB m = runb_merge(e16, o16);
    const RunB lo32 = runb_swap(m, true, false), hi32 = runb_swap(m, true, true);    // rows (0|1) and (2|3)
    return runb_merge(lo32, hi32);
}

// BF16 decision under the error bounds: certain iff the best row's upper
// bound is below every other row's lower bound.  Every lane of the point
// computes it.  When certain, the lane of row r.wq -- the one whose chunk
// store wrote the best group's bound, so that the two stores keep their
// order -- replaces that bound by the best group's second (bm2), and the
// lane of row 0 writes the point's state; otherwise the point is reported
// uncertain with U* (an upper bound on its true nearest distance).
__device__ __forceinline__ void decide_bf16(const ProbDev &P, int pid, bool dense, int a, float minnc, const RunB &r,
                                            float sdd, bool &moved, bool &amb, int &win, float &umin)
{
    const float Ub = root_hi(r.bu), Ls = root_lo(r.sec);
    amb = !(Ub < Ls) || r.bs < 0;
    moved = false;
    win = -1;
    umin = Ub;
    if (amb) return;
    const int q = lane_id() >> 4;
    if (q == r.wq) {
        const float sv = store_lb(root_lo(r.bm2), P.Sgd[r.bg]);
        if (P.lb16) P.lbh[(size_t)pid * P.gs + r.bg] = lb16_enc(sv, P.lbsc[1]);
        else P.lb[(size_t)pid * P.gs + r.bg] = sv;
    }
    if (q != 0) return;
    win = r.bs;
    PointState nsv;
    nsv.a = win;
    nsv.ga = pack_ga(P.slot_group[win], r.og);
    nsv.u = store_u(Ub, P.Scd[win]);
    nsv.p = store_lb(fminf(minnc, Ls), sdd);
    P.st[pid] = nsv;
    moved = win != (dense ? -1 : a);
}

// ============================================================ dense (iteration 1)
template <int DMAX>
__device__ __forceinline__ void b_dense_f32(const ProbDev &P, const int bid_, const int nblk_)
{
    const int lane = lane_id();
    const int wpb = blockDim.x / WAVE;
    const double eps2 = eps2_direct(P.d);
    const float sdd = P.Sdud[1];
    const long long ntiles = (P.n + WAVE - 1) / WAVE;
    unsigned long long n_moved = 0;
    for (long long tl = (long long)bid_ * wpb + threadIdx.x / WAVE; tl < ntiles;
         tl += (long long)nblk_ * wpb) {
        const long long idx = tl * WAVE + lane;
        const bool act = idx < P.n;
        const int pid = act ? (int)idx : 0;
        float x[DMAX];
#pragma unroll
        for (int i = 0; i < DMAX; ++i) x[i] = (act && i < P.d) ? P.X[(size_t)pid * P.d + i] : 0.f;
        Run r;
        run_init(r);
        float *lbrow = P.lb + (size_t)pid * P.gs;
        for (int g4 = 0; g4 < P.g; g4 += 4) {
            float outv[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int gg = 0; gg < 4; ++gg) {
                const int g = g4 + gg;
                if (g >= P.g) break;
                const Best3 gb = direct_group<DMAX>(P, g, x);
                if (act) {
                    outv[gg] = store_lb(dist_lo(gb.m1, eps2), P.Sgd[g]);
                    run_fold(P, r, gb, g);
                }
            }
            if (act) *(float4 *)(lbrow + g4) = make_float4(outv[0], outv[1], outv[2], outv[3]);
        }
        bool moved = false;
        if (act) moved = finish_f32(P, pid, true, -1, -1, false, KP_INF, KP_INF, KP_INF, r, eps2, sdd);
        n_moved += (unsigned long long)__popcll(__ballot(moved));
        const long long em = wave_append(&P.ctr[CTR_MV], moved);
        if (em >= 0) {
            P.mv_pt[em] = pid;
            P.mv_old[em] = -1;
            P.mv_new[em] = P.st[pid].a;
        }
    }
    if (lane == 0 && n_moved) atomicAdd(&P.ctr[CTR_MOVED], n_moved);
    if (bid_ == 0 && threadIdx.x == 0) {
        atomicAdd(&P.ctr[CTR_PAIRS], (unsigned long long)P.n * (unsigned long long)P.g);
        atomicAdd(&P.ctr[CTR_DIST], (unsigned long long)P.n * (unsigned long long)P.k);
    }
}
template <int DMAX>
__global__ __launch_bounds__(256) void k_dense_f32(ProbDev P)
{
    b_dense_f32<DMAX>(P, (int)blockIdx.x, (int)gridDim.x);
}
template <int DMAX>
__global__ __launch_bounds__(256) void kb_dense_f32(const ProbDev *__restrict__ probs, const int *__restrict__ tab, int count)
{
    const int pi = batch_problem(tab, count);
    const ProbDev P = probs[pi];
    b_dense_f32<DMAX>(P, (int)blockIdx.x - tab[pi], tab[pi + 1] - tab[pi]);
}


// ================================================ group-level filter (phase 1)
// One wave per tile of 64 consecutive entries of the sorted L1 (lane = point
// of the tile).  Every group bound of each point is tested against the
// point's upper bound (brought forward by its centroid's drift); the point's
// own group always stays open, so that the distance kernel recomputes the
// distance to the current centroid.  For each group open for some point of
// the tile, (group, 64-bit point mask) is appended to the tile's list; the
// distance kernel (phase 2) visits only those groups.  Per point it leaves
// ub and the smallest bound of the closed groups.
//
// The bound rows pass through LDS in chunks of 32 groups: lanes over the
// groups of two points on the way in (contiguous row runs, all loads of a
// chunk in flight together), lane = point on the way out.
constexpr int GT_WAVES = 4;
constexpr int GT_CH = 32;             // groups per LDS chunk
constexpr int GT_LD = GT_CH + 1;      // LDS row pitch (bank-conflict free)

__device__ __forceinline__ void b_group_test(const ProbDev &P, const int bid_, const int nblk_)
{
    __shared__ float stage[GT_WAVES][WAVE * GT_LD];
    const int lane = lane_id();
    const int wv = threadIdx.x / WAVE;
    float *sm = stage[wv];
    const long long count = list_len(P, CTR_L1);
    const long long ntiles = (count + WAVE - 1) / WAVE;
    const int half = lane >> 5, col = lane & 31;
    unsigned long long n_pairs = 0, n_visits = 0, n_closed = 0;
    for (long long tl = (long long)bid_ * GT_WAVES + wv; tl < ntiles; tl += (long long)nblk_ * GT_WAVES) {
        const long long idx = tl * WAVE + lane;
        const bool act = idx < count;
        const int pid = act ? clamp_pid(P, P.L1s[idx]) : 0;
        float ubt = KP_INF, minnc = KP_INF;
        int ga = -1;
        bool anyb = false;   // some group open by its bound (own group included)
        if (act) {
            const PointState s = P.st[pid];
            const int a = clamp_slot(P, s.a);
            ga = P.slot_group[a];
            ubt = ub_now(s.u, P.Scu[a]);
        }
        int cnt = 0;
        int4 *lst = P.tlist + (size_t)tl * P.g;
        for (int g0 = 0; g0 < P.g; g0 += GT_CH) {
            const int gw = min(GT_CH, P.g - g0);
            // in: row chunks of the tile's points, two points per step; every
            // load is issued before the first store (no branch between them)
            float rv[WAVE / 2];
            const int cc = min(col, gw - 1);
#pragma unroll
            for (int p0 = 0; p0 < WAVE; p0 += 2) {
                const int pp = __shfl(pid, p0 + half);   // inactive points carry pid 0
                rv[p0 / 2] = P.lb[(size_t)pp * P.gs + g0 + cc];
            }
#pragma unroll
            for (int p0 = 0; p0 < WAVE; p0 += 2) sm[(p0 + half) * GT_LD + col] = rv[p0 / 2];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // out: lane = point
            for (int j = 0; j < gw; ++j) {
                const int g = g0 + j;
                const float sgu = P.Sgu[g];
                const float v = act ? sm[lane * GT_LD + j] : 0.f;
                const bool byb = act && group_open(ubt, sgu, v);
                const bool cand = byb || (act && g == ga);
                anyb = anyb || byb;
                const unsigned long long m = __ballot(cand);
                if (m) {
                    if (lane == 0) lst[cnt] = make_int4(g, (int)(unsigned)m, (int)(unsigned)(m >> 32), 0);
                    ++cnt;
                    n_pairs += (unsigned long long)__popcll(m);
                }
                if (act && !cand) minnc = fminf(minnc, v - sgu);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (lane == 0) P.tcnt[tl] = cnt;
        n_visits += (unsigned long long)cnt;
        n_closed += (unsigned long long)__popcll(__ballot(act && !anyb));
        if (act) {
            P.ps4[idx] = make_float4(ubt, f_dn(minnc), 0.f, 0.f);
            P.psf[idx] = 1;
        }
    }
    if (lane == 0 && n_pairs) atomicAdd(&P.ctr[CTR_PAIRS], n_pairs);
    if (lane == 0 && n_visits) atomicAdd(&P.ctr[CTR_VISITS], n_visits);
    block_add_closed(P, n_closed);
}
__global__ __launch_bounds__(WAVE * GT_WAVES) void k_group_test(ProbDev P)
{
    b_group_test(P, (int)blockIdx.x, (int)gridDim.x);
}
__global__ __launch_bounds__(WAVE * GT_WAVES) void kb_group_test(const ProbDev *__restrict__ probs, const int *__restrict__ tab, int count)
{
    const int pi = batch_problem(tab, count);
    const ProbDev P = probs[pi];
    b_group_test(P, (int)blockIdx.x - tab[pi], tab[pi + 1] - tab[pi]);
}


// ======================================= group-level filter (BF16 mode)
// One workgroup per tile of 64 sorted L1 positions -- the distance kernel's
// tile -- with wave w on positions 16 w .. 16 w + 15.  Each point's group
// bounds are tested against its upper bound brought to this iteration: lane
// (point p, quad q) reads groups g0 + 16 q .. +15 of p's bound row as one
// 64-byte run.  The point's own group always stays open.  Writes, per
// position, the smallest bound of the closed groups (rounded down) and, per
// tile, the visit list of the distance kernel: every group open for some
// point of the tile, in group order, with the four waves' 16-bit point masks
// (g, m0 | m1 << 16, m2 | m3 << 16, 0), and its length.
template <bool LB16>   // bounds stored as FP16 codes
__device__ __forceinline__ void b_gfilter(const ProbDev &P, const int bid_, const int nblk_)
{
    __shared__ float gsu[GMAX_BF16];
    __shared__ unsigned short msk[2][4][WAVE];   // round r: wave w's point mask of group g0 + t
    for (int i = threadIdx.x; i < P.g; i += blockDim.x) gsu[i] = P.Sgu[i];
    for (int i = P.g + threadIdx.x; i < ((P.g + 3) & ~3); i += blockDim.x) gsu[i] = 0.f;   // float4 tail
    __syncthreads();
    const int lane = lane_id(), pt = lane & 15, quad = lane >> 4;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const long long count = list_len(P, CTR_L1);
    const long long ntiles = (count + 63) / 64;
    const float lsc = P.lbsc[0];
    constexpr bool lb16 = LB16;
    int rb = 0;   // mask buffer, alternating over every round of the launch
    unsigned long long n_closed = 0;
    for (long long tl = bid_; tl < ntiles; tl += nblk_) {   // uniform per workgroup
        const long long pos = tl * 64 + 16 * wv + pt;
        const bool in = pos < count;
        int pid = 0, ga = -1;
        float ubt = KP_INF;
        if (in) {
            const int4 e = P.L1x[pos];
            pid = clamp_pid(P, e.x);
            ubt = __int_as_float(e.z);
            ga = min(max(e.w, 0), P.g - 1);
        }
        const float *lbrow = P.lb + (size_t)pid * P.gs;
        const uint16_t *lbrow16 = P.lbh + (size_t)pid * P.gs;
        int4 *vis = P.tlist + (size_t)tl * P.g;
        float cm = KP_INF;
        int nv = 0;
        bool anyb = false;   // some group of this lane's 16 open by its bound (own group included)
        for (int g0 = 0; g0 < P.g; g0 += WAVE, rb ^= 1) {
            const int gq = g0 + 16 * quad;
            float v[16], sg[16];
            if constexpr (lb16) {
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    const int gi = gq + 8 * i;   // gs is padded to 8
                    const uint4 h = (in && gi < P.g) ? *(const uint4 *)(lbrow16 + gi) : make_uint4(0u, 0u, 0u, 0u);
                    const unsigned hw[4] = {h.x, h.y, h.z, h.w};
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        v[8 * i + 2 * q] = lb16_dec((unsigned short)(hw[q] & 0xFFFFu), lsc);
                        v[8 * i + 2 * q + 1] = lb16_dec((unsigned short)(hw[q] >> 16), lsc);
                    }
                }
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int gi = gq + 4 * i;
                    const float4 v4 = (in && gi < P.g) ? *(const float4 *)(lbrow + gi) : make_float4(0.f, 0.f, 0.f, 0.f);
                    v[4 * i] = v4.x;
                    v[4 * i + 1] = v4.y;
                    v[4 * i + 2] = v4.z;
                    v[4 * i + 3] = v4.w;
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int gi = gq + 4 * i;   // the LDS table is padded to 4
                const bool ok = in && gi < P.g;
                const float4 s4 = ok ? *(const float4 *)(gsu + gi) : make_float4(0.f, 0.f, 0.f, 0.f);
                sg[4 * i] = s4.x;
                sg[4 * i + 1] = s4.y;
                sg[4 * i + 2] = s4.z;
                sg[4 * i + 3] = s4.w;
            }
            unsigned bits = 0u;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int g = gq + j;
                const bool cand = in && g < P.g;
                const bool byb = cand && group_open(ubt, sg[j], v[j]);
                const bool open = byb || (cand && g == ga);
                anyb = anyb || byb;
                bits |= open ? 1u << j : 0u;
                cm = (cand && !open) ? fminf(cm, v[j] - sg[j]) : cm;   // rounded down once below
            }
            // transposed: lane t gets this wave's point mask of group g0 + t
            unsigned long long mine = 0ull;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const unsigned long long bj = __ballot((bits >> j) & 1u);
                if (pt == j) mine = bj;
            }
            msk[rb][wv][lane] = (unsigned short)((mine >> (16 * quad)) & 0xFFFFu);
            // one barrier per round: a buffer is rewritten two rounds later,
            // after every wave has passed the barrier of the round between
            __syncthreads();
            const unsigned m0 = msk[rb][0][lane], m1 = msk[rb][1][lane], m2 = msk[rb][2][lane],
                           m3 = msk[rb][3][lane];
            const bool open = g0 + lane < P.g && (m0 | m1 | m2 | m3) != 0u;
            const unsigned long long om = __ballot(open);
            if (wv == 0 && open)
                vis[nv + __popcll(om & ((1ull << lane) - 1ull))] =
                    make_int4(g0 + lane, (int)(m0 | (m1 << 16)), (int)(m2 | (m3 << 16)), 0);
            nv += __popcll(om);
        }
        cm = fminf(cm, __shfl_xor(cm, 16));
        cm = fminf(cm, __shfl_xor(cm, 32));
        if (in && quad == 0) P.minnc[pos] = f_dn(cm);
        if (wv == 0 && lane == 0) P.tcnt[tl] = nv;
        // points of this wave with every group closed by its bound
        const unsigned long long ob = __ballot(anyb), ib = __ballot(in);
        n_closed += (unsigned long long)__popcll(ib & ~(ob | ob >> 16 | ob >> 32 | ob >> 48) & 0xFFFFull);
    }
    block_add_closed(P, n_closed);
}
template <bool LB16>
__global__ __launch_bounds__(256) void k_gfilter(ProbDev P) { b_gfilter<LB16>(P, (int)blockIdx.x, (int)gridDim.x); }
template <bool LB16>
__global__ __launch_bounds__(256) void kb_gfilter(const ProbDev *__restrict__ probs, const int *__restrict__ tab,
                                                  int count)
{
    const int pi = batch_problem(tab, count);
    const ProbDev P = probs[pi];
    b_gfilter<LB16>(P, (int)blockIdx.x - tab[pi], tab[pi + 1] - tab[pi]);
}

// ================================================== distance kernels (phase 2)
constexpr int TF_STAGE = 1024;   // floats of centroid rows staged per wave (4 KB)

// Wave-local hand-off through LDS: the compiler keeps the accesses on either
// side in order, and a wave's LDS operations complete in issue order.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Copies n4 (1 <= n4 <= TF_STAGE / 4) 16-byte pieces from src into this
// wave's LDS region dst, all lanes taking part.  Every load is issued before
// the first store; lanes past n4 repeat the last piece (same address, same
// value), so there is no branch between the loads.
__device__ __forceinline__ void stage_rows(float *dst, const float *__restrict__ src, int n4, int lane)
{
    static_assert(TF_STAGE == 16 * WAVE, "four pieces per lane");
    const float4 *s4 = (const float4 *)src;
    float4 *d4 = (float4 *)dst;
    const int i0 = min(lane, n4 - 1), i1 = min(lane + WAVE, n4 - 1), i2 = min(lane + 2 * WAVE, n4 - 1),
              i3 = min(lane + 3 * WAVE, n4 - 1);
    const float4 v0 = s4[i0], v1 = s4[i1], v2 = s4[i2], v3 = s4[i3];
    wave_lds_sync();   // the previous rows have been read
    d4[i0] = v0;
    d4[i1] = v1;
    d4[i2] = v2;
    d4[i3] = v3;
    wave_lds_sync();
}

template <int DMAX>
__device__ __forceinline__ void b_tile_f32(const ProbDev &P, const int bid_, const int nblk_)
{
    static_assert(DMAX <= TF_STAGE / 8, "a staged batch holds at least eight rows");
    __shared__ __align__(16) float crows[4][TF_STAGE];   // launches have at most four waves
    const int lane = lane_id();
    const int wpb = blockDim.x / WAVE;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);   // the tile and its visits are uniform
    const double eps2 = eps2_direct(P.d);
    const float sdd = P.Sdud[1];
    const long long count = list_len(P, CTR_L1);
    const long long ntiles = (count + WAVE - 1) / WAVE;
    float *cw = crows[wv];
    const int mrow = TF_STAGE / P.ldc;   // rows per staged batch (ldc <= DMAX)
    unsigned long long n_dist = 0, n_moved = 0;
    for (long long tl = (long long)bid_ * wpb + wv; tl < ntiles; tl += (long long)nblk_ * wpb) {
        const long long idx = tl * WAVE + lane;
        const bool in = idx < count;
        const int flags = in ? P.psf[idx] : 0;
        const bool act = flags & 1, a_sep = flags & 2;
        if (__ballot(act) == 0ull) continue;
        const int pid = in ? clamp_pid(P, P.L1s[idx]) : 0;
        const float4 q = in ? P.ps4[idx] : make_float4(0.f, 0.f, 0.f, 0.f);
        const float d2a = q.w, lbe_a = q.z, minnc = q.y;
        const float ubt = q.x;   // ub brought to this iteration
        const int a = act ? clamp_slot(P, P.st[pid].a) : 0;
        const int ga = P.slot_group[a];
        float x[DMAX];
#pragma unroll
        for (int i = 0; i < DMAX; ++i) x[i] = (act && i < P.d) ? P.X[(size_t)pid * P.d + i] : 0.f;
        Run r;
        run_init(r);
        if (a_sep) {
            r.bd = d2a;
            r.bs = a;
        }
        float *lbrow = P.lb + (size_t)pid * P.gs;
        const int cnt = min(max(P.tcnt[tl], 0), P.g);
        const int4 *lst = P.tlist + (size_t)tl * P.g;
        // each visit's bound of this lane's point is loaded one visit ahead
        auto vis_of = [&](int k, unsigned long long &m) {
            int4 e = lst[k];
            e.x = min(max(e.x, 0), P.g - 1);
            m = (unsigned long long)(unsigned)e.y | ((unsigned long long)(unsigned)e.z << 32);
            return e.x;
        };
        const bool lf = P.lf != 0;
        unsigned long long mn = 0ull;
        int gn = cnt > 0 ? vis_of(0, mn) : 0;
        float vn = (lf && cnt > 0 && ((mn >> lane) & 1ull)) ? lbrow[gn] : 0.f;
        int s0n = P.gstart[gn], nsn = P.gsize[gn];   // the next visit's members, also loaded ahead
        for (int k = 0; k < cnt; ++k) {
            const int g = gn;
            const unsigned long long m = mn;
            const float vrow = vn;
            const int s0 = s0n, ns = nsn;
            if (k + 1 < cnt) {
                gn = vis_of(k + 1, mn);
                vn = (lf && ((mn >> lane) & 1ull)) ? lbrow[gn] : 0.f;
                s0n = P.gstart[gn];
                nsn = P.gsize[gn];
            }
            const bool mine = (m >> lane) & 1ull;
            // Local filter (kp_tuning.local_filter): member j of g lies at
            // least lb(x, g) brought forward plus slk[j] from x (the bound
            // moved by g's largest drift, the member by its own); it is
            // skipped when that exceeds ub for every point of the wave that
            // visits g, and is never a visiting point's own centroid.  Skipped
            // members enter the group's bound and lbp with that lower bound,
            // never the search for the nearest.
            const float lbn = (mine && lf) ? lb_now(vrow, P.Sgu[g]) : 0.f;
            Best3 gb = {KP_INF, -1, KP_INF};
            float lk = KP_INF;
            int ncomp = 0;
            // the group's rows are contiguous: staged in LDS a batch at a time
            // (one memory latency per batch), then read from there
            for (int b0 = 0; b0 < ns; b0 += mrow) {
                const int mb = min(mrow, ns - b0);
                stage_rows(cw, P.c32 + (size_t)(s0 + b0) * P.ldc, mb * P.ldc / 4, lane);
                for (int rr = 0; rr < mb; ++rr) {
                    const int j = s0 + b0 + rr;
                    const float L = lf ? f_dn(lbn + P.slk[j]) : 0.f;
                    if (lf && __ballot(mine && !(j != a && L > ubt)) == 0ull) {
                        lk = fminf(lk, L);
                        continue;
                    }
                    ++ncomp;
                    const float v = direct_d2<DMAX>(x, cw + rr * P.ldc, P.ldc);
                    if (v < gb.m1) {
                        gb.m2 = gb.m1;
                        gb.m1 = v;
                        gb.s1 = j;
                    } else {
                        gb.m2 = fminf(gb.m2, v);
                    }
                }
            }
            n_dist += (unsigned long long)__popcll(m) * (unsigned long long)ncomp;
            if (mine) {
                gb.m2 = fminf(gb.m2, lk < KP_INF ? f_dn(lk * lk) : KP_INF);   // squared, rounded down
                lbrow[g] = store_lb(fminf(dist_lo(gb.m1, eps2), lk), P.Sgd[g]);
                run_fold(P, r, gb, g);
                r.lk = fminf(r.lk, lk);
            }
        }
        bool moved = false;
        if (act) moved = finish_f32(P, pid, false, a, ga, a_sep, d2a, lbe_a, minnc, r, eps2, sdd);
        n_moved += (unsigned long long)__popcll(__ballot(moved));
        const long long em = wave_append(&P.ctr[CTR_MV], moved);
        if (em >= 0) {
            P.mv_pt[em] = pid;
            P.mv_old[em] = a;
            P.mv_new[em] = P.st[pid].a;
        }
    }
    if (lane == 0 && n_dist) atomicAdd(&P.ctr[CTR_DIST], n_dist);
    if (lane == 0 && n_moved) atomicAdd(&P.ctr[CTR_MOVED], n_moved);
}
template <int DMAX>
__global__ __launch_bounds__(256) void k_tile_f32(ProbDev P)
{
    b_tile_f32<DMAX>(P, (int)blockIdx.x, (int)gridDim.x);
}
template <int DMAX>
__global__ __launch_bounds__(256) void kb_tile_f32(const ProbDev *__restrict__ probs, const int *__restrict__ tab, int count)
{
    const int pi = batch_problem(tab, count);
    const ProbDev P = probs[pi];
    b_tile_f32<DMAX>(P, (int)blockIdx.x - tab[pi], tab[pi + 1] - tab[pi]);
}


// ---------------------------------------------- workgroup of 64 positions
// Four waves; wave w holds positions 16 w .. 16 w + 15 of the tile in its B
// operand.  The workgroup walks one list of chunks, the union of its waves'
// visits: each chunk's A operand is staged in LDS once for the four waves,
// the next chunk loading while the current one is on the matrix cores.  A
// staged chunk keeps fragment (part, ks) of lane l at a[part * KS + ks][l]
// (one conflict-free 16-byte read per lane and fragment), then the norms.
template <int KS>
struct ChunkStage {
    bf16x8 a[2 * KS][WAVE];
    float4 cn[8];   // the rows' Q: ||c_j||^2, or ||c_j - r||^2 relative to an anchor r;
                    // then (cn[4 + q], read as nr[q]) their N_j >= ||c~_j|| (0 for the first row, padding)
    float2 wt;      // the chunk's (W, c W^2) for the bounds
};
// The anchor of a tile's estimates: slot a (-1: none, r = 0) and this
// thread's coordinate t of c32_a (0 beyond the row), which it subtracts from
// the chunk's first row when staging it.
struct Anchor {
    int a;
    float rt;
};
// One visit of a tile: a group, its first slot, size and rounded-down drift
// sum (copied from the group tables when the list is loaded, so that a
// chunk step reads its description in one LDS access), and the four waves'
// 16-bit point masks.
struct Visit {
    int g, s0, ns;
    float sgd;
    unsigned short m[4];
};
template <int KS>
struct BlockLds {
    ChunkStage<KS> st[2];
    Visit vis[GMAX_BF16];           // the tile's visits (filtered), or every group in order (dense, serving)
    // wide rows (two workgroups per CU, so LDS is not the limit): the group
    // tables kept in LDS too, for the visit list's lookups of each tile
    static constexpr int GT = KS >= 6 ? GMAX_BF16 : 1;
    int gst[GT], gsz[GT];
    float gsd[GT];
    float ar[32 * KS];              // the tile's anchor row (filtered iterations with anchors)
};
template <int KS>
struct StageRegs {
    bf16x8 r[(2 * KS * WAVE + 255) / 256];
    float4 c;  // threads 0..3: Q of rows 4t..4t+3; threads 4..7: N of rows 4(t-4)..
    float2 wt;
    float w;   // with an anchor: coordinate t of the chunk's first row, c32_f
};

// Loads of the chunk at slot0 into this thread's staging registers.  Every
// thread issues the same loads whatever the sizes (entries past the chunk
// repeat one inside it), so that the memory counters of the pipelined loop
// below stay exact.  With an anchor the rows' Q come from its row of the
// table Qt and the chunk's first row is loaded in FP32 (one coordinate per
// thread) to be staged relative to the anchor.
template <int KS>
__device__ __forceinline__ void stage_load(const ProbDev &P, int slot0, StageRegs<KS> &s, const Anchor &anc)
{
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < (2 * KS * WAVE + 255) / 256; ++i) {
        const int e = (t + 256 * i) % (2 * KS * WAVE);
        const int f = e / WAVE, l = e % WAVE;   // f = part * KS + ks
        const uint16_t *base = (f >= KS) ? P.cbl : P.cb;
        const int ks = f % KS;
        s.r[i] = *(const bf16x8 *)(base + (size_t)(slot0 + (l & 15)) * P.ldb + 32 * ks + 8 * (l >> 4));
    }
    const int ch = slot0 / CHUNK;
    const float *qrow = anc.a >= 0 ? P.Qt + (size_t)anc.a * P.kg : P.cn;
    s.c = *(const float4 *)((t & 4) ? P.nrel + slot0 + 4 * (t & 3) : qrow + slot0 + 4 * (t & 3));
    if (anc.a >= 0) {
        s.wt = P.Wa[(size_t)anc.a * P.nch + ch];
        s.w = P.c32[(size_t)slot0 * P.ldc + min(t, P.ldc - 1)];
    } else {
        s.wt = P.Wu[ch];
        s.w = 0.f;
    }
}
template <int KS>
__device__ __forceinline__ void stage_store(ChunkStage<KS> &S, const StageRegs<KS> &s, const Anchor &anc,
                                            int ldc)
{
    const int t = threadIdx.x;
    // every fragment of a thread with t % 16 == 0 is a row-0 fragment (e = t
    // + 256 i keeps e % 64 = t % 64): with an anchor those are restaged below
    if (!(anc.a >= 0 && (t & 15) == 0)) {
#pragma unroll
        for (int i = 0; i < (2 * KS * WAVE + 255) / 256; ++i) {
            const int e = t + 256 * i;
            if ((2 * KS * WAVE) % 256 == 0 || e < 2 * KS * WAVE) S.a[e / WAVE][e % WAVE] = s.r[i];
        }
    }
    if (anc.a >= 0 && t < 32 * KS) {
        // coordinate t of w~ = fl(c32_f - r) into row 0: fragment ks = t / 32,
        // lane 16 (t % 32 / 8), element t % 8, split as the other rows
        const float w = (t < ldc ? s.w : 0.f) - anc.rt;
        const __bf16 h = (__bf16)w;
        const __bf16 l = (__bf16)(w - (float)h);
        const int ks = t / 32, lane = 16 * ((t & 31) >> 3), el = t & 7;
        S.a[ks][lane][el] = h;
        S.a[KS + ks][lane][el] = l;
    }
    if (t < 8) S.cn[t] = s.c;   // cn[0..3], then nr[0..3] (adjacent)
    if (t == 0) S.wt = s.wt;
}

// Row 0's product of this lane's point (lane p, element 0) in every lane of
// the point: two swaps move it from row 0 to rows 2, then 1 and 3.
__device__ __forceinline__ float row0_bcast(float x)
{
    const auto a = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    const auto b = __builtin_amdgcn_permlane16_swap(a[0], a[0], false, false);
    return __uint_as_float(b[0]);
}
// The estimates themselves, clamped at 0 (a squared distance is >= 0, so the
// clamp only moves an estimate toward the true value).  Row 0 of the chunk
// is its first slot f: its product is x~.w~; every other row j gives x~.c~_j,
// to which x~.w~ is added (the rows are stored relative to row 0).
__device__ __forceinline__ void chunk_est(const f32x4 &hh, const f32x4 &lo, float4 c4, float xnp, float (&v)[4])
{
    const float s0 = row0_bcast(hh[0] + lo[0]);
    const bool q0 = lane_id() < 16;
    const float cnv[4] = {c4.x, c4.y, c4.z, c4.w};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const float sj = hh[r] + lo[r];
        const float S = (q0 && r == 0) ? sj : sj + s0;
        v[r] = fmaxf(fmaf(-2.f, S, xnp + cnv[r]), 0.f);
    }
}
// The bound e_j of each of this lane's rows from the point's (b A, a A^2),
// the chunk's (W, c W^2) and the rows' N_j: e_j = E0 + N_j (h + c N_j).
__device__ __forceinline__ void chunk_eta(float2 pt, float2 wt, float4 n4, float (&e)[4])
{
    const float E0 = fmaf(pt.x, wt.x, pt.y + wt.y);
    const float h = fmaf(ETA3_C2, wt.x, pt.x);
    e[0] = fmaf(n4.x, fmaf(ETA3_C, n4.x, h), E0);
    e[1] = fmaf(n4.y, fmaf(ETA3_C, n4.y, h), E0);
    e[2] = fmaf(n4.z, fmaf(ETA3_C, n4.z, h), E0);
    e[3] = fmaf(n4.w, fmaf(ETA3_C, n4.w, h), E0);
}
// This lane's partial Key3 over its four rows (slots 4 (l >> 4) .. +3).
__device__ __forceinline__ Key3 chunk_key3(const f32x4 &hh, const f32x4 &lo, float4 c4, float4 n4, float xnp, float2 pt,
                                           float2 wt)
{
    const unsigned base = 4u * (unsigned)(lane_id() >> 4);
    float v[4], e[4];
    chunk_est(hh, lo, c4, xnp, v);
    chunk_eta(pt, wt, n4, e);
    unsigned k[4];
    float u[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const float L = fmaxf(v[r] - e[r], 0.f);
        u[r] = v[r] + e[r];
        k[r] = (__float_as_uint(L) & ~15u) | (base + (unsigned)r);
    }
    const Key3 p = k[0] < k[1] ? Key3{k[0], k[1], u[0]} : Key3{k[1], k[0], u[1]};
    const Key3 q = k[2] < k[3] ? Key3{k[2], k[3], u[2]} : Key3{k[3], k[2], u[3]};
    return key3_merge(p, q);
}

// The two accumulators of a staged chunk against this wave's points: hh the
// leading products, lo the two correction products (accumulated apart and
// added once, so that no product waits on the one issued just before it;
// every element still sums at most ldb + 1 terms, which the bound covers).
template <int KS>
__device__ __forceinline__ void chunk_acc(const ChunkStage<KS> &S, const PtFrag<KS> &b, f32x4 &hh, f32x4 &lo)
{
    const int lane = lane_id();
    hh = f32x4{0.f, 0.f, 0.f, 0.f};
    lo = f32x4{0.f, 0.f, 0.f, 0.f};
    f32x4 l2 = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const bf16x8 ah = S.a[ks][lane], al = S.a[KS + ks][lane];
        hh = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, b.h[ks], hh, 0, 0, 0);
        lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, b.h[ks], lo, 0, 0, 0);
        l2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, b.l[ks], l2, 0, 0, 0);
    }
    lo[0] += l2[0];
    lo[1] += l2[1];
    lo[2] += l2[2];
    lo[3] += l2[3];
}
template <int KS>
__device__ __forceinline__ Key3 chunk_lds(const ChunkStage<KS> &S, const PtFrag<KS> &b, float xnp, float2 pt)
{
    f32x4 hh, lo;
    chunk_acc<KS>(S, b, hh, lo);
    const int q = lane_id() >> 4;
    return chunk_key3(hh, lo, S.cn[q], S.cn[4 + q], xnp, pt, S.wt);
}

// Chunks of a tile's visits 0 .. nv-1 (workgroup-uniform); src(k, g, m, s0,
// ns, sgd) gives visit k's group, this wave's point mask, first slot, size
// (>= 1) and rounded-down drift sum.
struct ChunkSeq {
    int k, c0, s0, ns;
    bool valid;
};
template <class Src>
__device__ __forceinline__ void seq_take(ChunkSeq &q, Src &src)
{
    int g, s0, ns;
    unsigned m;
    float sgd;
    src(q.k, g, m, s0, ns, sgd);
    q.s0 = s0;
    q.ns = ns;
    q.c0 = 0;
}
template <class Src>
__device__ __forceinline__ void seq_begin(ChunkSeq &q, int nv, Src &src)
{
    q.k = 0;
    q.c0 = q.s0 = q.ns = 0;
    q.valid = nv > 0;
    if (q.valid) seq_take(q, src);
}
template <class Src>
__device__ __forceinline__ void seq_next(ChunkSeq &q, int nv, Src &src)
{
    q.c0 += CHUNK;
    if (q.c0 >= q.ns) {
        if (++q.k < nv) seq_take(q, src);
        else q.valid = false;
    }
}
// Advance a load cursor; past the last chunk it stays on it.
template <class Src>
__device__ __forceinline__ void seq_next_load(ChunkSeq &q, int nv, Src &src)
{
    if (q.c0 + CHUNK < q.ns) {
        q.c0 += CHUNK;
    } else if (q.k + 1 < nv) {
        ++q.k;
        seq_take(q, src);
    }
}

// The workgroup's visits 0 .. nv-1 from src.  Every thread of the workgroup
// calls it.  Per chunk, each lane reduces its four rows of its point to a
// Key3 partial (a wave with no point in the visit skips the products and
// calls skip(), which issues the same memory operations).
//   TRANS (every group is one chunk): the partials of four consecutive
//   chunks are reduced and spread together (key3_scatter4), and
//   fold4(p0..p3, m0..m3, n) is called with row q of lanes finishing chunk
//   q of the n (<= 4) pending ones, m_q its description.
//   Otherwise every chunk is reduced over the four rows (key3_fold_all) and
//   fold1(g, m, slot0, first, sgd, key3) called with every lane holding the
//   chunk's result for its point.
// note(g, m, nreal, first) sees every chunk (wave-uniform counts).
//
// DEPTH chunks are in flight: chunk i is read from LDS while chunks
// i+1 .. i+DEPTH-1 are loading into registers; after chunk i the loads of
// chunk i+DEPTH are issued and chunk i+1 goes to LDS.  With DEPTH = 1 the
// next chunk's loads are issued before the current chunk's work.
struct ChunkMeta {
    int g, slot0;
    unsigned m;
    float sgd;
};
// Wave-uniform values read from LDS, moved to scalar registers.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ unsigned uni(unsigned v) { return (unsigned)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ float uni(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }

// The description of chunk q of four (field by field: a selection of whole
// structures would take their addresses).
__device__ __forceinline__ ChunkMeta meta_of(int q, ChunkMeta m0, ChunkMeta m1, ChunkMeta m2, ChunkMeta m3)
{
    ChunkMeta r;
    r.g = q == 0 ? m0.g : (q == 1 ? m1.g : (q == 2 ? m2.g : m3.g));
    r.slot0 = q == 0 ? m0.slot0 : (q == 1 ? m1.slot0 : (q == 2 ? m2.slot0 : m3.slot0));
    r.m = q == 0 ? m0.m : (q == 1 ? m1.m : (q == 2 ? m2.m : m3.m));
    r.sgd = q == 0 ? m0.sgd : (q == 1 ? m1.sgd : (q == 2 ? m2.sgd : m3.sgd));
    return r;
}
template <int KS, int DEPTH, bool TRANS, class Src, class Note, class Fold1, class Fold4, class Skip>
__device__ __forceinline__ void block_visits(const ProbDev &P, BlockLds<KS> &L, int nv, Src src,
                                             const PtFrag<KS> &b, float xnp, float2 pt, const Anchor &anc,
                                             Note note, Fold1 fold1, Fold4 fold4, Skip skip)
{
    if (nv <= 0) return;
    ChunkSeq cp, ld;
    seq_begin(cp, nv, src);
    ld = cp;
    StageRegs<KS> R[DEPTH];
#pragma unroll
    for (int k = 0; k < DEPTH; ++k) {
        stage_load<KS>(P, ld.s0 + ld.c0, R[k], anc);
        seq_next_load(ld, nv, src);
    }
    stage_store<KS>(L.st[0], R[0], anc, P.ldc);
    __syncthreads();
    int buf = 0;
    // the pending chunks' partials and descriptions (named registers: the
    // slot of a step is a constant of the unrolled loop)
    Key3 p0 = key3_empty(), p1 = key3_empty(), p2 = key3_empty(), p3 = key3_empty();
    ChunkMeta m0{0, 0, 0u, 0.f}, m1 = m0, m2 = m0, m3 = m0;
    auto work = [&](int slot) {
        int g, s0, ns;
        unsigned m;
        float sgd;
        src(cp.k, g, m, s0, ns, sgd);
        note(g, m, min(CHUNK, cp.ns - cp.c0), cp.c0 == 0);
        Key3 t = key3_empty();
        if (m) t = chunk_lds<KS>(L.st[buf], b, xnp, pt);
        else if (!TRANS) skip();
        if (TRANS) {
            const ChunkMeta mt{g, cp.s0 + cp.c0, m, sgd};
            if (slot == 0) {
                p0 = t;
                m0 = mt;
            } else if (slot == 1) {
                p1 = t;
                m1 = mt;
            } else if (slot == 2) {
                p2 = t;
                m2 = mt;
            } else {
                p3 = t;
                m3 = mt;
            }
        } else if (m) {
            fold1(g, m, cp.s0 + cp.c0, cp.c0 == 0, sgd, key3_fold_all(t));
        }
    };
    constexpr int U = TRANS ? (DEPTH == 3 ? 12 : 4) : DEPTH;
    for (;;) {
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const int k = i % DEPTH, slot = i % 4;
            if (DEPTH == 1) {
                stage_load<KS>(P, ld.s0 + ld.c0, R[0], anc);
                seq_next_load(ld, nv, src);
                work(slot);
            } else {
                work(slot);
                stage_load<KS>(P, ld.s0 + ld.c0, R[k], anc);
                seq_next_load(ld, nv, src);
            }
            stage_store<KS>(L.st[buf ^ 1], R[(k + 1) % DEPTH], anc, P.ldc);
            __syncthreads();
            seq_next(cp, nv, src);
            buf ^= 1;
            if (TRANS && slot == 3) fold4(p0, p1, p2, p3, m0, m1, m2, m3, 4);
            if (!cp.valid) {
                if (TRANS && slot != 3) fold4(p0, p1, p2, p3, m0, m1, m2, m3, slot + 1);
                return;
            }
        }
    }
}

// BF16 mode, one workgroup per tile of 64 positions.  DENSE (iteration 1):
// the positions are the points and every group is visited.  Otherwise the
// positions are entries of the sorted L1 and the workgroup visits every
// group that the group filter left open for some point of the tile (the
// points' own groups always are).  Per point: the decision under the error
// bound, or the entry that sends it to the FP32 recheck.
template <int KS, bool DENSE, int DEPTH>
__device__ __forceinline__ void b_blk64(const ProbDev &P, const int bid_, const int nblk_)
{
    __shared__ BlockLds<KS> L;
    const int lane = lane_id(), pt = lane & 15, quad = lane >> 4, wv = threadIdx.x / WAVE;
    const Eta3 ek = mfma_eta3_coef(P.ldb);
    const float sdd = P.Sdud[1];
    const bool track_og = P.nk1 > P.kg;   // the L1 order uses the nearest other group
    const bool lb16 = P.lb16 != 0;        // bounds as FP16 codes
    const bool anchored = !DENSE && P.anch != 0;   // estimates relative to the tile's anchor centroid
    const float linv = P.lbsc[1];
    float *sink = P.sink + 16 * (bid_ % SINK_SLOTS);
    const long long count = DENSE ? P.n : list_len(P, CTR_L1);
    const long long ntiles = (count + 63) / 64;
    if (DENSE) {
        for (int i = threadIdx.x; i < P.g; i += blockDim.x) {
            Visit &d = L.vis[i];
            d.g = i;
            d.s0 = P.gstart[i];
            d.ns = P.gsize[i];
            d.sgd = P.Sgd[i];
        }
        __syncthreads();
    } else if (KS >= 6) {
        for (int i = threadIdx.x; i < P.g; i += blockDim.x) {
            L.gst[i] = P.gstart[i];
            L.gsz[i] = P.gsize[i];
            L.gsd[i] = P.Sgd[i];
        }
        __syncthreads();
    }
    unsigned long long n_dist = 0, n_pairs = 0, n_visits = 0, n_moved = 0;
    // sorted entry of this lane's position in the tile after the one being
    // fetched, loaded one tile ahead
    int2 nxt = make_int2(0, 0);   // point and slot of the entry (its first half)
    if (!DENSE) {
        const long long i0 = (long long)bid_ * 64 + 16 * wv + pt;
        if (i0 < count) nxt = *(const int2 *)(P.L1x + i0);
    }
    // A tile's inputs, fetched while the previous tile is finished: this
    // lane's point, old slot, norm, closed-group bound and FP32 coordinates,
    // and (filtered) the length of the tile's visit list and this thread's
    // entry of it; with anchors, the tile's anchor slot (that of its first
    // entry: the entries are sorted by slot) and this thread's coordinate of
    // the anchor's row.
    int f_pid = 0, f_a = -1, f_nv = 0, f_anc = -1;
    float f_xn = 0.f, f_minnc = KP_INF, f_rt = 0.f;
    float f_v[KS][8];
    int4 f_ent = make_int4(0, 0, 0, 0);
    auto fetch = [&](long long tf) {
        const long long ix = tf * 64 + 16 * wv + pt;
        const bool ok = ix < count;
        f_pid = ok && DENSE ? (int)ix : 0;
        f_a = -1;
        if (!DENSE) {
            const int2 e = nxt;
            const long long inext = ix + 64ll * nblk_;
            if (inext < count) nxt = *(const int2 *)(P.L1x + inext);
            if (ok) {
                f_pid = clamp_pid(P, e.x);
                f_a = clamp_slot(P, e.y);
            }
        }
        f_xn = (ok && !anchored) ? P.xn[f_pid] : 0.f;
        f_minnc = (!DENSE && ok) ? P.minnc[ix] : KP_INF;
        load_rows16<KS>(P, f_pid, ok, f_v);
        if (!DENSE && tf < ntiles) {
            f_nv = P.tcnt[tf];
            if ((int)threadIdx.x < P.g) f_ent = P.tlist[(size_t)tf * P.g + threadIdx.x];
            if (anchored) {
                f_anc = clamp_slot(P, P.L1x[tf * 64].y);
                f_rt = (int)threadIdx.x < P.ldc ? P.c32[(size_t)f_anc * P.ldc + threadIdx.x] : 0.f;
            }
        }
    };
    if (bid_ < ntiles) fetch(bid_);
    for (long long tl = bid_; tl < ntiles; tl += nblk_) {   // uniform per workgroup
        const long long idx = tl * 64 + 16 * wv + pt;
        const bool in = idx < count;
        const int pid = f_pid, a = f_a;
        const float minnc = f_minnc;
        const Anchor anc = {anchored ? f_anc : -1, anchored ? f_rt : 0.f};
        const unsigned inm = (unsigned)__ballot(in) & 0xFFFFu;   // this wave's points
        PtFrag<KS> b;
        float xnp = f_xn;
        RunB r;
        runb_init(r);
        float gmin = KP_INF;   // squared lower bound of the group being visited, so far
        float2 eA;
        unsigned t_pairs = 0u, t_dist = 0u;   // this tile's counts (< 2^32)
        auto note = [&](int, unsigned m, int nreal, bool first) {
            const unsigned pm = (unsigned)__popc(m);
            t_pairs += first ? pm : 0u;
            t_dist += pm * (unsigned)nreal;
        };
        // a visited group's bound of this lane's point, offset form, rounded
        // down; lanes with nothing to write send the store to the sink slot
        auto put_lb = [&](bool mine, int g, float l, float sgd) {
            const float lbv = dn_nonneg(root_lo(l) + sgd);
            if (lb16) {
                uint16_t *dst = mine ? P.lbh + (size_t)pid * P.gs + g : (uint16_t *)sink;
                *dst = lb16_enc(lbv, linv);
            } else {
                float *dst = mine ? P.lb + (size_t)pid * P.gs + g : sink;
                *dst = lbv;
            }
        };
        // every lane holds the chunk's result for its point (groups of more
        // than one chunk); one unconditional store per chunk
        auto fold1 = [&](int g, unsigned m, int slot0, bool first, float sgd, const Key3 &kk) {
            const bool mine = (m >> pt) & 1u;
            const float l1 = key_value(kk.k1), l2 = key_value(kk.k2);
            const float gprev = first ? KP_INF : gmin;
            gmin = fminf(gprev, l1);
            runb_fold(r, mine, l1, kk.u1, slot0 + (int)(kk.k1 & 15u), l2, g, gprev, track_og);
            r.wq = 0;   // every lane folds every chunk; the stores are row 0's
            put_lb(mine && quad == 0, g, gmin, sgd);
        };
        // row q of lanes finishes chunk q of the n pending ones (every group
        // is one chunk, so l1 is the group's bound); one store per lane
        auto fold4 = [&](Key3 p0, Key3 p1, Key3 p2, Key3 p3, ChunkMeta m0, ChunkMeta m1, ChunkMeta m2, ChunkMeta m3,
                         int n) {
            const Key3 kk = key3_scatter4(p0, p1, p2, p3);
            const ChunkMeta mq = meta_of(quad, m0, m1, m2, m3);
            const bool mine = quad < n && ((mq.m >> pt) & 1u);
            const float l1 = key_value(kk.k1), l2 = key_value(kk.k2);
            runb_fold(r, mine, l1, kk.u1, mq.slot0 + (int)(kk.k1 & 15u), l2, mq.g, KP_INF, track_og);
            put_lb(mine, mq.g, l1, mq.sgd);
        };
        auto skip = [&]() { *(uint16_t *)sink = 0; };
        // every group is one chunk, and rows of 128 or more coordinates:
        // with fewer, a chunk step has few products and the fold's exchanges
        // cost more than the chunk results kept by every lane (measured at
        // d = 16..64: 84 ms against 105 ms per 25 batched iterations)
        const bool trans = KS >= 4 && P.maxgs <= CHUNK;
        auto visits = [&](int nv, auto src) {
            if (trans) {
                block_visits<KS, DEPTH, true>(P, L, nv, src, b, xnp, eA, anc, note, fold1, fold4, skip);
                r = runb_allreduce(r);
            } else {
                block_visits<KS, DEPTH, false>(P, L, nv, src, b, xnp, eA, anc, note, fold1, fold4, skip);
            }
        };
        if (DENSE) {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) split8(f_v[ks], b.h[ks], b.l[ks]);
            eA = mfma_eta3_pt(ek, mfma_eta3_a(xnp));
            // every group, in order
            auto src = [&](int k, int &g, unsigned &m, int &s0, int &ns, float &sgd) {
                g = k;
                m = inm;
                s0 = uni(L.vis[k].s0);
                ns = uni(L.vis[k].ns);
                sgd = uni(L.vis[k].sgd);
            };
            n_visits += wv == 0 ? (unsigned long long)P.g : 0ull;
            visits(P.g, src);
        } else {
            // the tile's visit list, written by the group filter (the first
            // entries fetched with the tile's inputs), and the anchor's row
            const int nv = min(max(f_nv, 0), P.g);
            const int4 *tv = P.tlist + (size_t)tl * P.g;
            for (int k = threadIdx.x; k < nv; k += blockDim.x) {
                const int4 v = k == (int)threadIdx.x ? f_ent : tv[k];
                Visit &d = L.vis[k];
                d.g = min(max(v.x, 0), P.g - 1);
                if constexpr (KS >= 6) {
                    d.s0 = L.gst[d.g];
                    d.ns = L.gsz[d.g];
                    d.sgd = L.gsd[d.g];
                } else {
                    d.s0 = P.gstart[d.g];
                    d.ns = P.gsize[d.g];
                    d.sgd = P.Sgd[d.g];
                }
                d.m[0] = (unsigned short)((unsigned)v.y & 0xFFFFu);
                d.m[1] = (unsigned short)((unsigned)v.y >> 16);
                d.m[2] = (unsigned short)((unsigned)v.z & 0xFFFFu);
                d.m[3] = (unsigned short)((unsigned)v.z >> 16);
            }
            if (anchored && (int)threadIdx.x < 32 * KS) L.ar[threadIdx.x] = anc.rt;
            __syncthreads();
            if (anchored) {
                // x~ = fl(x - c_a) and its squared norm (FP64, rounded once)
                double sq = 0.0;
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    const float4 r0 = *(const float4 *)&L.ar[32 * ks + 8 * quad];
                    const float4 r1 = *(const float4 *)&L.ar[32 * ks + 8 * quad + 4];
                    const float rr[8] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const float xv = f_v[ks][j] - rr[j];
                        f_v[ks][j] = xv;
                        sq = fma((double)xv, (double)xv, sq);
                    }
                }
                sq += __shfl_xor(sq, 16);
                sq += __shfl_xor(sq, 32);
                xnp = (float)sq;
            }
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) split8(f_v[ks], b.h[ks], b.l[ks]);
            eA = mfma_eta3_pt(ek, mfma_eta3_a(xnp));
            auto src = [&](int k, int &g, unsigned &m, int &s0, int &ns, float &sgd) {
                const Visit &v = L.vis[k];
                g = uni(v.g);
                m = uni((unsigned)v.m[wv]);
                s0 = uni(v.s0);
                ns = uni(v.ns);
                sgd = uni(v.sgd);
            };
            n_visits += wv == 0 ? (unsigned long long)nv : 0ull;
            visits(nv, src);
        }
        n_pairs += t_pairs;
        n_dist += t_dist;
        // the next tile's loads are in flight while this one is finished
        fetch(tl + nblk_);
        bool moved = false, amb = false;
        int win = -1;
        const long long pos = DENSE ? (long long)pid : idx;
        if (in) {
            float umin = KP_INF;
            decide_bf16(P, pid, DENSE, a, minnc, r, sdd, moved, amb, win, umin);
            amb = amb && quad == 0;   // one entry per point
            // the recheck's inputs: the BF16 best slot and U*
            if (amb) P.ps4[pos] = make_float4(__int_as_float(r.bs), 0.f, umin, 0.f);
        }
        n_moved += (unsigned long long)__popcll(__ballot(moved));
        // moved points: compact list for the centroid update
        const long long em = wave_append(&P.ctr[CTR_MV], moved);
        if (em >= 0) {
            P.mv_pt[em] = pid;
            P.mv_old[em] = a;
            P.mv_new[em] = win;
        }
        // uncertain points: compact list of positions for the FP32 recheck
        const long long q3 = wave_append(&P.ctr[CTR_L3], amb);
        if (q3 >= 0) P.L3[q3] = (int)pos;
    }
    if (lane == 0) {
        if (n_dist) atomicAdd(&P.ctr[CTR_DIST], n_dist);
        if (n_pairs) atomicAdd(&P.ctr[CTR_PAIRS], n_pairs);
        if (n_visits) atomicAdd(&P.ctr[CTR_VISITS], n_visits);
        if (n_moved) atomicAdd(&P.ctr[CTR_MOVED], n_moved);
    }
}
// Three workgroups per CU (three waves per SIMD) are asked of the register
// allocation up to KS = 4; wider rows get two (three would spill).  The
// batched form keeps the default (its problem lookup would spill).
template <int KS, bool DENSE, int DEPTH>
__global__ __launch_bounds__(256, KS <= 4 ? 3 : 2) void k_blk64(ProbDev P)
{
    b_blk64<KS, DENSE, DEPTH>(P, (int)blockIdx.x, (int)gridDim.x);
}
template <int KS, bool DENSE, int DEPTH>
__global__ __launch_bounds__(256) void kb_blk64(const ProbDev *__restrict__ probs, const int *__restrict__ tab, int count)
{
    const int pi = batch_problem(tab, count);
    const ProbDev P = probs[pi];
    b_blk64<KS, DENSE, DEPTH>(P, (int)blockIdx.x - tab[pi], tab[pi + 1] - tab[pi]);
}


// ================================================================ recheck
// Eight lanes (a team) per uncertain point, 32 points per workgroup.
// Candidates: every group whose lower bound is <= U*, an upper bound on the
// point's true nearest distance; every other centroid is provably farther
// than the nearest one.  Their distances are recomputed in FP32 direct form
// on the FP32 point, which the team holds in registers: lane t owns
// coordinates 4t + 32j .. 4t + 32j + 3, sums its d/8 terms in coordinate
// order, then a three-level tree combines the lanes (relative error below
// eps2_direct).  The point is decided on those values (lowest original index
// on exact ties).  The candidate rows come straight from L2: staging the
// union of a workgroup's candidate groups in LDS was measured slower (its
// barriers serialise the teams, and most teams idle in most groups).
constexpr int RT = 8;                 // lanes per point
constexpr int RMAX = 64;              // candidate groups kept in LDS per point

__device__ __forceinline__ float team_sum(float v)
{
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    return v;
}
__device__ __forceinline__ float team_min(float v)
{
    v = fminf(v, __shfl_xor(v, 1));
    v = fminf(v, __shfl_xor(v, 2));
    v = fminf(v, __shfl_xor(v, 4));
    return v;
}
__device__ __forceinline__ int wave_max_i(int v)
{
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

template <int NV>   // float4 per lane: d <= 32 * NV
__device__ __forceinline__ void team_load(float4 (&c4)[NV], const float *__restrict__ c, int ldc, int t)
{
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const int i = 4 * t + 32 * j;
        c4[j] = i < ldc ? *(const float4 *)(c + i) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
}
template <int NV>
__device__ __forceinline__ float team_dist(const float4 (&x)[NV], const float4 (&c4)[NV])
{
    float acc = 0.f;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const float t0 = x[j].x - c4[j].x, t1 = x[j].y - c4[j].y, t2 = x[j].z - c4[j].z, t3 = x[j].w - c4[j].w;
        acc = fmaf(t0, t0, acc);
        acc = fmaf(t1, t1, acc);
        acc = fmaf(t2, t2, acc);
        acc = fmaf(t3, t3, acc);
    }
    return team_sum(acc);
}
template <int NV>
__device__ __forceinline__ float team_d2(const float4 (&x)[NV], const float *__restrict__ c, int ldc, int t)
{
    float4 c4[NV];
    team_load<NV>(c4, c, ldc, t);
    return team_dist<NV>(x, c4);
}

template <int NV, bool LB16>   // LB16: bounds stored as FP16 codes
__device__ __forceinline__ void b_recheck(const ProbDev &P, const int bid_, const int nblk_)
{
    constexpr int TPB = 256 / RT;   // teams per workgroup
    __shared__ int rg[TPB][RMAX];
    __shared__ float rm1[TPB][RMAX], rm2[TPB][RMAX];
    __shared__ float sgu[GMAX_BF16];
    const int lane = lane_id();
    const int t = lane & (RT - 1);
    const int team = threadIdx.x / RT;
    const double eps2 = eps2_direct(P.d);
    const float sdd = P.Sdud[1];
    const bool dense = P.ctr[CTR_DENSE] != 0;
    const long long n3 = list_len(P, CTR_L3);   // uncertain positions, listed by the distance kernel
    const long long mv0 = list_len(P, CTR_MV);  // update entries the distance kernel wrote before these
    const int last_pos = (int)(positions(P) - 1);  // counters read once: other waves update their line
    const long long nteams = (long long)nblk_ * TPB;
    const long long trips = (n3 + nteams - 1) / nteams;   // the same for every lane of the grid
    const float lsc = P.lbsc[0], linv = P.lbsc[1];
    constexpr bool lb16 = LB16;
    for (int g = threadIdx.x; g < P.g; g += blockDim.x) sgu[g] = P.Sgu[g];
    __syncthreads();
    const unsigned long long tlanes = 0xFFull << (lane & ~(RT - 1));   // this team's lanes
    const unsigned long long below = tlanes & ((1ull << lane) - 1ull);  // ... below this lane
    unsigned long long n_moved = 0;
    for (long long it = 0; it < trips; ++it) {
        const long long e0 = it * nteams + (long long)bid_ * TPB;
        const long long e3 = e0 + team;
        const bool live = e3 < n3;
        if (__ballot(live) == 0ull) continue;   // past the end of the list for this wave's eight teams
        const long long e = live ? (long long)max(min(P.L3[e3], last_pos), 0) : 0;
        const int pid = live ? (dense ? (int)e : clamp_pid(P, P.L1x[e].x)) : 0;
        const int olda = (live && !dense) ? clamp_slot(P, P.st[pid].a) : -1;
        const float4 pin = live ? P.ps4[e] : make_float4(0.f, 0.f, 0.f, 0.f);
        float4 x[NV];
        const float *xrow = P.X + (size_t)pid * P.d;
        if ((P.d & 3) == 0 && ((uintptr_t)P.X & 15) == 0) {   // rows of whole, aligned float4
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                const int i = 4 * t + 32 * j;
                x[j] = (live && i < P.d) ? *(const float4 *)(xrow + i) : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        } else {
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                const int i = 4 * t + 32 * j;
                float v[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = (live && i + q < P.d) ? xrow[i + q] : 0.f;
                x[j] = make_float4(v[0], v[1], v[2], v[3]);
            }
        }
        // candidate threshold: the smaller of U* and an upper bound on the
        // FP32 direct-form distance to the BF16 pass's best centroid (either
        // bounds the nearest distance from above; the second has no BF16
        // error in it)
        const int bslot = clamp_slot(P, __float_as_int(pin.x));
        const float umin = fminf(pin.z, dist_hi(team_d2<NV>(x, P.c32 + (size_t)bslot * P.ldc, P.ldc, t), eps2));
        float *lbrow = P.lb + (size_t)pid * P.gs;
        uint16_t *lbrow16 = P.lbh + (size_t)pid * P.gs;
        // groups that may hold the nearest centroid, in ascending order: the
        // team reads the bounds in blocks of 64 groups, lane t groups
        // 64 j + 8 t .. 64 j + 8 t + 7 (16 bytes of FP16 codes or 32 of
        // FP32), SB blocks in flight
        float minnr = KP_INF;
        int nR = 0;
        const int ng = live ? P.g : 0;
        const int nb64 = (P.g + 63) / 64;
        constexpr int SB = 2;
        for (int j0 = 0; j0 < nb64; j0 += SB) {
            uint4 lv[SB][2];
            const uint4 z4 = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
            for (int b = 0; b < SB; ++b) {
                const int gq = 64 * (j0 + b) + 8 * t;   // the row is padded to a multiple of 8
                if constexpr (lb16) {
                    lv[b][0] = gq < ng ? *(const uint4 *)(lbrow16 + gq) : z4;
                    lv[b][1] = z4;
                } else {
                    lv[b][0] = gq < ng ? *(const uint4 *)(lbrow + gq) : z4;
                    lv[b][1] = gq + 4 < ng ? *(const uint4 *)(lbrow + gq + 4) : z4;
                }
            }
#pragma unroll
            for (int b = 0; b < SB; ++b) {
                const int gq = 64 * (j0 + b) + 8 * t;
                const unsigned hw[8] = {lv[b][0].x, lv[b][0].y, lv[b][0].z, lv[b][0].w,
                                        lv[b][1].x, lv[b][1].y, lv[b][1].z, lv[b][1].w};
                unsigned in8 = 0u;
                int nbelow = 0, nteam = 0;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int g = gq + q;
                    bool inR = false;
                    if (g < ng) {
                        const float v = lb16 ? lb16_dec((unsigned short)(hw[q >> 1] >> (16 * (q & 1))), lsc)
                                             : __uint_as_float(hw[q]);
                        const float lbe = lb_now(v, sgu[g]);
                        inR = lbe <= umin;
                        if (!inR) minnr = fminf(minnr, lbe);
                    }
                    in8 |= inR ? 1u << q : 0u;
                    const unsigned long long m = __ballot(inR);
                    nbelow += __popcll(m & below);
                    nteam += __popcll(m & tlanes);
                }
                int pos = nR + nbelow;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    if ((in8 >> q) & 1u) {
                        if (pos < RMAX) rg[team][pos] = gq + q;
                        ++pos;
                    }
                }
                nR += nteam;
            }
        }
        minnr = team_min(minnr);
        // more than RMAX candidate groups: examine every group (rare)
        const bool overflow = nR > RMAX;
        const int nscan = overflow ? ng : nR;
        const int nscan_w = wave_max_i(nscan);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        float bd = KP_INF, ov = KP_INF;
        int bs = -1, bgr = -1, og = -1;
        for (int i = 0; i < nscan_w; ++i) {
            const bool on = i < nscan;
            const int g = on ? (overflow ? i : rg[team][i]) : 0;
            const int s0 = P.gstart[g], ns = on ? P.gsize[g] : 0;
            const int ns_w = wave_max_i(ns);
            float m1 = KP_INF, m2 = KP_INF;
            int s1 = -1;
            constexpr int BATCH = NV <= 4 ? 4 : 2;   // candidates whose rows are in flight together
            for (int r = 0; r < ns_w; r += BATCH) {
                float4 c4[BATCH][NV];
#pragma unroll
                for (int q = 0; q < BATCH; ++q)
                    team_load<NV>(c4[q], P.c32 + (size_t)(s0 + (r + q < ns ? r + q : 0)) * P.ldc, P.ldc, t);
#pragma unroll
                for (int q = 0; q < BATCH; ++q) {
                    const float v = team_dist<NV>(x, c4[q]);
                    if (r + q < ns) {
                        // slots need not ascend by original index (a chunk's
                        // first slot is its medoid): exact ties go to the lower one
                        if (before(P, v, s0 + r + q, m1, s1)) {
                            m2 = m1;
                            m1 = v;
                            s1 = s0 + r + q;
                        } else {
                            m2 = fminf(m2, v);
                        }
                    }
                }
            }
            if (on) {
                if (!overflow && t == 0) {
                    rm1[team][i] = m1;
                    rm2[team][i] = m2;
                }
                if (before(P, m1, s1, bd, bs)) {
                    if (g != bgr) {
                        ov = bd;
                        og = bgr;
                    }
                    bd = m1;
                    bs = s1;
                    bgr = g;
                } else if (g != bgr && m1 < ov) {
                    ov = m1;
                    og = g;
                }
            }
        }
        if (bs < 0) bs = olda >= 0 ? olda : 0;   // unreachable: the provisional winner's group is a candidate
        const int gbest = P.slot_group[bs];
        // lower bounds of the examined groups
        float minr = KP_INF;
        if (!overflow) {
            for (int i = t; i < nR; i += RT) {
                const int g = rg[team][i];
                const float lbv = dist_lo(g == gbest ? rm2[team][i] : rm1[team][i], eps2);
                const float sv = store_lb(lbv, P.Sgd[g]);
                if (lb16) lbrow16[g] = lb16_enc(sv, linv);
                else lbrow[g] = sv;
                minr = fminf(minr, lbv);
            }
        } else {
            // second pass: the minimum of every group except the winner
            const int nw2 = wave_max_i(overflow ? ng : 0);
            for (int i = 0; i < nw2; ++i) {
                const bool on = overflow && i < ng;
                const int g = on ? i : 0;
                const int s0 = P.gstart[g], ns = on ? P.gsize[g] : 0;
                const int ns_w = wave_max_i(ns);
                float m = KP_INF;
                for (int r = 0; r < ns_w; ++r) {
                    const bool ok = r < ns && (s0 + r) != bs;
                    const float v = team_d2<NV>(x, P.c32 + (size_t)(s0 + (r < ns ? r : 0)) * P.ldc, P.ldc, t);
                    if (ok) m = fminf(m, v);
                }
                if (on) {
                    const float lbv = dist_lo(m, eps2);
                    const float sv = store_lb(lbv, P.Sgd[g]);
                    if (t == 0 && lb16) lbrow16[g] = lb16_enc(sv, linv);
                    if (t == 0 && !lb16) lbrow[g] = sv;
                    minr = fminf(minr, lbv);
                }
            }
        }
        minr = team_min(minr);
        if (!live) continue;
        const float lbp = fminf(minnr, minr);
        if (t == 0) {
            PointState nsv;
            nsv.a = bs;
            nsv.u = store_u(dist_hi(bd, eps2), P.Scd[bs]);
            nsv.p = store_lb(lbp, sdd);
            nsv.ga = pack_ga(gbest, og);
            P.st[pid] = nsv;
            n_moved += bs != olda ? 1ull : 0ull;
            // the centroid update's entry of this point, after the entries
            // the distance kernel listed (-1: did not move)
            const long long em = mv0 + e3;
            P.mv_pt[em] = pid;
            P.mv_old[em] = olda;
            P.mv_new[em] = bs != olda ? bs : -1;
        }
    }
    // one atomic per lane that decided points (lane 0 of each team)
    if (n_moved) atomicAdd(&P.ctr[CTR_MOVED], n_moved);
}
template <int NV, bool LB16>
__global__ __launch_bounds__(256) void k_recheck(ProbDev P)
{
    b_recheck<NV, LB16>(P, (int)blockIdx.x, (int)gridDim.x);
}
template <int NV, bool LB16>
__global__ __launch_bounds__(256) void kb_recheck(const ProbDev *__restrict__ probs, const int *__restrict__ tab, int count)
{
    const int pi = batch_problem(tab, count);
    const ProbDev P = probs[pi];
    b_recheck<NV, LB16>(P, (int)blockIdx.x - tab[pi], tab[pi + 1] - tab[pi]);
}


// ========================================================= centroid update
// Entries of the centroid update: the points the distance kernels decided
// and moved (a compact list), then one entry per rechecked point (mv_new = -1
// when it did not move) -- M in all.  e < M adds point mv_pt[e] to slot
// mv_new[e]; M <= e < 2M subtracts point mv_pt[e-M] from slot mv_old[e-M].
// Points that had no slot before (mv_old = -1, the dense iteration)
// contribute no subtraction.
__device__ __forceinline__ long long update_len(const ProbDev &P)
{
    const long long m = list_len(P, CTR_MV) + list_len(P, CTR_L3);
    return m < (long long)P.n ? m : (long long)P.n;
}
__device__ __forceinline__ int entry_key(const ProbDev &P, long long e, long long M)
{
    const long long q = e < M ? e : e - M;
    const int kn = P.mv_new[q];
    if (kn < 0) return -1;
    const int k = e < M ? kn : P.mv_old[q];
    return k < 0 ? -1 : clamp_slot(P, k);
}

__device__ __forceinline__ void b_hist(const ProbDev &P, const int bid_, const int nblk_)
{
    __shared__ int h[HIST_LDS];
    const long long M = update_len(P);
    const long long E = 2 * M;
    const bool lds = P.kg <= HIST_LDS;
    if (lds)
        for (int i = threadIdx.x; i < P.kg; i += blockDim.x) h[i] = 0;
    __syncthreads();
    for (long long e = (long long)bid_ * blockDim.x + threadIdx.x; e < E;
         e += (long long)nblk_ * blockDim.x) {
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
__global__ __launch_bounds__(256) void k_hist(ProbDev P)
{
    b_hist(P, (int)blockIdx.x, (int)gridDim.x);
}
__global__ __launch_bounds__(256) void kb_hist(const ProbDev *__restrict__ probs, const int *__restrict__ tab, int count)
{
    const int pi = batch_problem(tab, count);
    const ProbDev P = probs[pi];
    b_hist(P, (int)blockIdx.x - tab[pi], tab[pi + 1] - tab[pi]);
}


__device__ __forceinline__ void b_scatter(const ProbDev &P, const int bid_, const int nblk_)
{
    __shared__ int h[HIST_LDS];
    __shared__ int base[HIST_LDS];
    const long long M = update_len(P);
    const long long E = 2 * M;
    const bool lds = P.kg <= HIST_LDS;
    const long long b0 = E * bid_ / nblk_, b1 = E * (bid_ + 1) / nblk_;
    if (!lds) {
        for (long long e = b0 + threadIdx.x; e < b1; e += blockDim.x) {
            const int key = entry_key(P, e, M);
            if (key < 0) continue;
            const int pos = atomicAdd(&P.cursor[key], 1);
            const int pid = clamp_pid(P, P.mv_pt[e < M ? e : e - M]);
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
        const int pid = clamp_pid(P, P.mv_pt[e < M ? e : e - M]);
        P.srt_pt[pos] = e < M ? pid : (int)((unsigned)pid | 0x80000000u);
        P.srt_key[pos] = key;
    }
}
__global__ __launch_bounds__(256) void k_scatter(ProbDev P)
{
    b_scatter(P, (int)blockIdx.x, (int)gridDim.x);
}
__global__ __launch_bounds__(256) void kb_scatter(const ProbDev *__restrict__ probs, const int *__restrict__ tab, int count)
{
    const int pi = batch_problem(tab, count);
    const ProbDev P = probs[pi];
    b_scatter(P, (int)blockIdx.x - tab[pi], tab[pi + 1] - tab[pi]);
}


// One wave per run of 64 sorted entries; lanes over coordinates.  Sums are
// FP64; a change of key flushes the run with FP64 atomics.
template <int DCH>
__device__ __forceinline__ void b_segsum(const ProbDev &P, const int bid_, const int nblk_)
{
    const int lane = lane_id();
    const long long M = update_len(P);
    const long long used = (long long)P.cursor[P.kg - 1];   // end of the last bin = entries sorted
    const long long E = used < 2 * M ? used : 2 * M;
    constexpr int SEG = DCH <= 2 ? 16 : (DCH <= 4 ? 8 : 2);   // sorted entries per wave and pass: their rows load together
    const long long nchunks = (E + SEG - 1) / SEG;
    const long long nw = (long long)nblk_ * (blockDim.x / WAVE);
    for (long long c = (long long)bid_ * (blockDim.x / WAVE) + threadIdx.x / WAVE; c < nchunks; c += nw) {
        const long long p0 = c * SEG;
        const int cnt = (int)((p0 + SEG < E) ? SEG : E - p0);
        // lane i < cnt holds entry p0 + i: its slot and (signed) point
        const int ekey = lane < cnt ? clamp_slot(P, P.srt_key[p0 + lane]) : 0;
        const int ept = lane < cnt ? P.srt_pt[p0 + lane] : 0;
        float xv[SEG][DCH];
#pragma unroll
        for (int i = 0; i < SEG; ++i) {
            const int v = __builtin_amdgcn_readlane(ept, i);
            const float *xr = P.X + (size_t)clamp_pid(P, v & 0x7FFFFFFF) * P.d;
#pragma unroll
            for (int j = 0; j < DCH; ++j) {
                const int dim = lane + WAVE * j;
                xv[i][j] = (i < cnt && dim < P.d) ? xr[dim] : 0.f;
            }
        }
        double acc[DCH];
#pragma unroll
        for (int j = 0; j < DCH; ++j) acc[j] = 0.0;
        int cacc = 0;
        int cur = __builtin_amdgcn_readlane(ekey, 0);
#pragma unroll
        for (int i = 0; i < SEG; ++i) {
            if (i >= cnt) break;
            const int key = __builtin_amdgcn_readlane(ekey, i);
            const bool neg = __builtin_amdgcn_readlane(ept, i) < 0;
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
#pragma unroll
            for (int j = 0; j < DCH; ++j) {
                const double x = (double)xv[i][j];
                acc[j] += neg ? -x : x;
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
template <int DCH>
__global__ __launch_bounds__(256) void k_segsum(ProbDev P)
{
    b_segsum<DCH>(P, (int)blockIdx.x, (int)gridDim.x);
}
template <int DCH>
__global__ __launch_bounds__(256) void kb_segsum(const ProbDev *__restrict__ probs, const int *__restrict__ tab, int count)
{
    const int pi = batch_problem(tab, count);
    const ProbDev P = probs[pi];
    b_segsum<DCH>(P, (int)blockIdx.x - tab[pi], tab[pi + 1] - tab[pi]);
}


// ======================================================= deterministic mode
// kp_tuning.deterministic replaces the three places where the order of
// floating-point or list work follows the order in which waves happen to run:
// the positions of the point-filter failures in L1 (one atomic per chunk),
// the order of equal keys in the counting sorts (LDS atomics) and the FP64
// atomic adds of the centroid update.  Each list is built in a fixed order
// instead, and the centroid sums are recomputed from all points in a fixed
// order.

// Exclusive scan of the per-chunk failure counts into their L1 offsets, and
// the list length (single workgroup of 1024).
__global__ __launch_bounds__(1024) void k_bf_scan(ProbDev P, int nchunks)
{
    __shared__ int part[1024];
    const int tid = threadIdx.x;
    const int per = (nchunks + 1023) / 1024;
    const int b = tid * per, e = min(nchunks, b + per);
    long long sum = 0;
    for (int i = b; i < e; ++i) sum += P.dcnt[i];
    part[tid] = (int)sum;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int v = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int run = part[tid] - (int)sum;
    for (int i = b; i < e; ++i) {
        P.doff[i] = run;
        run += P.dcnt[i];
    }
    if (tid == 1023) P.ctr[CTR_L1] = (unsigned long long)part[1023];
}

// Lanes of the wave whose key equals this lane's (only active lanes; 0 for an
// inactive lane): the key compared bit by bit with one ballot per bit.
__device__ __forceinline__ unsigned long long match_key(int key, int nbits, bool act)
{
    unsigned long long m = __ballot(act);
    for (int b = 0; b < nbits; ++b) {
        const bool bit = (key >> b) & 1;
        const unsigned long long bb = __ballot(act && bit);
        m &= bit ? bb : ~bb;
    }
    return act ? m : 0ull;
}

// Stable counting sort of E items by key (0 <= key < 2^nbits), block b of
// SS_NB one-wave blocks owning items [E b / SS_NB, E (b + 1) / SS_NB).
// hist: counts per (key, block) at key * SS_NB + block (zeroed before);
// after the scan they are the blocks' first positions per key, and the
// scatter advances them.  Each (key, block) counter is touched by one wave
// only, in item order, so every position is fixed by the keys and the input
// order alone.
template <class Src>
__device__ __forceinline__ void b_ss_hist(const Src &src, long long E, int nbits, int *__restrict__ hist)
{
    const int b = blockIdx.x, lane = lane_id();
    const long long lo = E * b / SS_NB, hi = E * (b + 1) / SS_NB;
    for (long long s0 = lo; s0 < hi; s0 += WAVE) {
        const long long i = s0 + lane;
        const bool act = i < hi;
        const int key = act ? src.key(i) : 0;
        const unsigned long long m = match_key(key, nbits, act);
        if (act && lane == __ffsll((long long)m) - 1) atomicAdd(&hist[(size_t)key * SS_NB + b], __popcll(m));
    }
}
template <class Src, class Dst>
__device__ __forceinline__ void b_ss_scatter(const Src &src, const Dst &dst, long long E, int nbits,
                                             int *__restrict__ cur)
{
    const int b = blockIdx.x, lane = lane_id();
    const long long lo = E * b / SS_NB, hi = E * (b + 1) / SS_NB;
    const unsigned long long below = (1ull << lane) - 1ull;
    for (long long s0 = lo; s0 < hi; s0 += WAVE) {
        const long long i = s0 + lane;
        const bool act = i < hi;
        const int key = act ? src.key(i) : 0;
        const unsigned long long m = match_key(key, nbits, act);
        const int leader = act ? __ffsll((long long)m) - 1 : lane;
        int base = 0;
        if (act && lane == leader) base = atomicAdd(&cur[(size_t)key * SS_NB + b], __popcll(m));
        base = __shfl(base, leader);
        if (act) dst.put((long long)base + __popcll(m & below), i, key);
    }
}

// Exclusive scan of the (key, block) table, L = nkeys * SS_NB entries, in three
// launches: per-workgroup totals, their scan, then each workgroup's part.
__global__ __launch_bounds__(256) void k_fill0(int *a, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        a[i] = 0;
}
__device__ __forceinline__ int block_sum_256(int v)
{
    __shared__ int red[4];
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    if (lane_id() == 0) red[threadIdx.x / WAVE] = v;
    __syncthreads();
    const int t = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
    return t;
}
__global__ __launch_bounds__(256) void k_ss_scan_part(const int *__restrict__ a, long long L, int *part)
{
    const long long lo = L * blockIdx.x / SS_SCAN_BLOCKS, hi = L * (blockIdx.x + 1) / SS_SCAN_BLOCKS;
    int s = 0;
    for (long long i = lo + threadIdx.x; i < hi; i += 256) s += a[i];
    s = block_sum_256(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}
__global__ __launch_bounds__(1024) void k_ss_scan_top(int *part)
{
    static_assert(SS_SCAN_BLOCKS == 1024, "one thread per part");
    __shared__ int sh[1024];
    const int tid = threadIdx.x;
    const int v = part[tid];
    sh[tid] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int w = tid >= o ? sh[tid - o] : 0;
        __syncthreads();
        sh[tid] += w;
        __syncthreads();
    }
    part[tid] = sh[tid] - v;
}
__global__ __launch_bounds__(256) void k_ss_scan_fin(int *a, long long L, const int *part)
{
    __shared__ int sh[256];
    const long long lo = L * blockIdx.x / SS_SCAN_BLOCKS, hi = L * (blockIdx.x + 1) / SS_SCAN_BLOCKS;
    const long long len = hi - lo;
    const long long per = (len + 255) / 256;
    const long long b = lo + threadIdx.x * per, e = min(hi, b + per);
    int s = 0;
    for (long long i = b; i < e; ++i) s += a[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const int w = (int)threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += w;
        __syncthreads();
    }
    int run = part[blockIdx.x] + sh[threadIdx.x] - s;
    for (long long i = b; i < e; ++i) {
        const int v = a[i];
        a[i] = run;
        run += v;
    }
}

// The sorts' item sources and destinations.
struct SrcL1 {   // L1 entries (deterministic order) keyed like the L1 order
    ProbDev P;
    __device__ int key(long long i) const
    {
        const int4 u = P.L1[i];
        return l1_key(P, clamp_slot(P, u.y), u.w);
    }
};
struct DstL1 {
    ProbDev P;
    __device__ void put(long long pos, long long i, int) const
    {
        const int4 u = P.L1[i];
        const int pid = clamp_pid(P, u.x), a = clamp_slot(P, u.y);
        if (P.prec) P.L1x[pos] = make_int4(pid, a, u.z, u.w & 0xFFFF);
        else P.L1s[pos] = pid;
    }
};
struct SrcPts {  // every point, keyed by its assigned slot
    ProbDev P;
    __device__ int key(long long i) const { return clamp_slot(P, P.st[i].a); }
};
struct DstPts {
    ProbDev P;
    __device__ void put(long long pos, long long i, int key) const
    {
        P.srt_pt[pos] = (int)i;
        P.srt_key[pos] = key;
    }
};
__global__ __launch_bounds__(64) void k_ss_hist_l1(ProbDev P)
{
    b_ss_hist(SrcL1{P}, list_len(P, CTR_L1), P.nb_l1, P.hist2);
}
__global__ __launch_bounds__(64) void k_ss_scatter_l1(ProbDev P)
{
    b_ss_scatter(SrcL1{P}, DstL1{P}, list_len(P, CTR_L1), P.nb_l1, P.hist2);
}
__global__ __launch_bounds__(64) void k_ss_hist_pts(ProbDev P) { b_ss_hist(SrcPts{P}, P.n, P.nb_slot, P.hist2); }
__global__ __launch_bounds__(64) void k_ss_scatter_pts(ProbDev P)
{
    b_ss_scatter(SrcPts{P}, DstPts{P}, P.n, P.nb_slot, P.hist2);
}

// Fixed-order centroid sums over the points sorted by (slot, index).  After
// the scatter, hist2[s * SS_NB + SS_NB - 1] is the end of slot s's segment.
__device__ __forceinline__ long long seg_end(const ProbDev &P, int s)
{
    return s < 0 ? 0 : (long long)P.hist2[(size_t)s * SS_NB + SS_NB - 1];
}
// One wave per piece of DS_PIECE sorted positions (lanes over coordinates).
// Each run of one slot inside the piece is summed in position order: a run
// that is the slot's whole segment is written to its sums; otherwise it is
// the piece's first run (it continues a segment from the previous piece) or
// its last run (the segment continues in the next), kept for k_dsum_fix.
template <int DCH>
__global__ __launch_bounds__(256) void k_dsum_piece(ProbDev P)
{
    const int lane = lane_id();
    const long long npieces = (P.n + DS_PIECE - 1) / DS_PIECE;
    const long long nw = (long long)gridDim.x * (blockDim.x / WAVE);
    for (long long pc = (long long)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE; pc < npieces; pc += nw) {
        const long long ps = pc * DS_PIECE, pe = min((long long)P.n, ps + DS_PIECE);
        long long pos = ps;
        while (pos < pe) {
            const int s = clamp_slot(P, P.srt_key[pos]);
            const long long ss = seg_end(P, s - 1), se = seg_end(P, s);
            const long long re = min(pe, se);
            double acc[DCH];
#pragma unroll
            for (int j = 0; j < DCH; ++j) acc[j] = 0.0;
            constexpr int U = DCH <= 4 ? 8 : 4;   // rows in flight
            for (long long q0 = pos; q0 < re; q0 += U) {
                float xv[U][DCH];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const bool ok = q0 + u < re;
                    const float *xr = P.X + (size_t)clamp_pid(P, ok ? P.srt_pt[q0 + u] : 0) * P.d;
#pragma unroll
                    for (int j = 0; j < DCH; ++j) {
                        const int dim = lane + WAVE * j;
                        xv[u][j] = (ok && dim < P.d) ? xr[dim] : 0.f;
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int j = 0; j < DCH; ++j) acc[j] += (double)xv[u][j];
            }
            double *out = (pos == ss && re == se) ? P.sums + (size_t)s * P.d
                          : (pos != ss) ? P.pfirst + (size_t)pc * P.d : P.plast + (size_t)pc * P.d;
#pragma unroll
            for (int j = 0; j < DCH; ++j) {
                const int dim = lane + WAVE * j;
                if (dim < P.d) out[dim] = acc[j];
            }
            pos = re;
        }
    }
}
// One wave per slot: the count, and the sum of a segment that spans pieces
// p0 < p1 as plast[p0] + pfirst[p0 + 1] + ... + pfirst[p1], in that order.
template <int DCH>
__global__ __launch_bounds__(256) void k_dsum_fix(ProbDev P)
{
    const int lane = lane_id();
    const int nw = gridDim.x * (blockDim.x / WAVE);
    for (int s = blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE; s < P.kg; s += nw) {
        const long long ss = seg_end(P, s - 1), se = seg_end(P, s);
        if (lane == 0) P.cnt[s] = (int)(se - ss);
        if (se <= ss) continue;
        const long long p0 = ss / DS_PIECE, p1 = (se - 1) / DS_PIECE;
        if (p0 == p1) continue;   // written whole by k_dsum_piece
        double acc[DCH];
#pragma unroll
        for (int j = 0; j < DCH; ++j) {
            const int dim = lane + WAVE * j;
            acc[j] = dim < P.d ? P.plast[(size_t)p0 * P.d + dim] : 0.0;
        }
        for (long long p = p0 + 1; p <= p1; ++p)
#pragma unroll
            for (int j = 0; j < DCH; ++j) {
                const int dim = lane + WAVE * j;
                if (dim < P.d) acc[j] += P.pfirst[(size_t)p * P.d + dim];
            }
#pragma unroll
        for (int j = 0; j < DCH; ++j) {
            const int dim = lane + WAVE * j;
            if (dim < P.d) P.sums[(size_t)s * P.d + dim] = acc[j];
        }
    }
}

// ================================================================ serving
// New query points assigned to a problem's current centroids with the
// iteration's decision rule -- the assignment step of Section 1 applied to
// points outside the training set.  BF16 mode: every group is visited as in
// the dense iteration, on tiles of 64 queries, and a query whose nearest
// centroid is certain under the error bound is labelled at once; the others
// are listed for an FP32 direct-form pass over every centroid.  FP32 mode:
// every query takes that pass.  Nothing of the problem's state is written.

// ||x||^2 of this lane's point from its 8 KS coordinates: FP64 squares summed
// over the four lanes of the point, rounded to FP32 once.
template <int KS>
__device__ __forceinline__ float norm_rows16(const float (&v)[KS][8])
{
    double s = 0.0;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int j = 0; j < 8; ++j) s = fma((double)v[ks][j], (double)v[ks][j], s);
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    return (float)s;
}

// ucnt[0], ucnt[1]: the two passes' uncertain-query counters; ucnt[2]: nq,
// the length of the list of every query (the first anchored pass reads it).
__global__ void k_serve_begin(unsigned long long *ucnt, long long nq)
{
    ucnt[0] = ucnt[1] = 0ull;
    ucnt[2] = (unsigned long long)nq;
}

// Serving's anchor of every query: the group whose chunk medoid (the first
// slot of its first chunk) has the smallest single-product BF16 estimate
// ||c_f||^2 - 2 xh.ch, written as that slot.  The choice only has to be
// near; the anchored passes that follow bound their own errors.  Tiles of 64
// queries (16 per wave); the medoid rows of 16 groups are staged in LDS per
// step, rows past g repeating the last group with +inf as norm.
template <int KS>
__global__ __launch_bounds__(256) void k_serve_pre(ProbDev P, const float *__restrict__ Q, long long nq,
                                                   int *__restrict__ anch)
{
    __shared__ bf16x8 A[KS][WAVE];
    __shared__ float cnv[16];
    const int lane = lane_id(), pt = lane & 15, quad = lane >> 4, wv = threadIdx.x / WAVE;
    const int t = threadIdx.x;
    ProbDev Pq = P;
    Pq.X = Q;
    const long long ntiles = (nq + 63) / 64;
    for (long long tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {   // uniform per workgroup
        const long long q = tl * 64 + 16 * wv + pt;
        const bool in = q < nq;
        float v[KS][8];
        load_rows16<KS>(Pq, in ? (int)q : 0, in, v);
        bf16x8 bh[KS];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            bf16x8 bl;
            split8(v[ks], bh[ks], bl);
        }
        float best = KP_INF;
        int bg = 0;
        for (int g0 = 0; g0 < P.g; g0 += 16) {
            __syncthreads();   // the previous step's reads of A are done
            for (int e = t; e < KS * WAVE; e += blockDim.x) {
                const int ks = e / WAVE, l = e % WAVE;
                const int slot = P.gstart[min(g0 + (l & 15), P.g - 1)];
                A[ks][l] = *(const bf16x8 *)(P.cb + (size_t)slot * P.ldb + 32 * ks + 8 * (l >> 4));
            }
            if (t < 16) cnv[t] = g0 + t < P.g ? P.cn[P.gstart[g0 + t]] : KP_INF;
            __syncthreads();
            f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[ks][lane], bh[ks], acc, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 4 * quad + r;
                const float e = fmaf(-2.f, acc[r], cnv[row]);
                if (e < best) {
                    best = e;
                    bg = g0 + row;
                }
            }
        }
        // the four lanes of a query hold disjoint rows
#pragma unroll
        for (int o = 16; o <= 32; o <<= 1) {
            const float ob = __shfl_xor(best, o);
            const int og = __shfl_xor(bg, o);
            if (ob < best || (ob == best && og < bg)) {
                best = ob;
                bg = og;
            }
        }
        if (in && quad == 0) anch[q] = P.gstart[min(max(bg, 0), P.g - 1)];
    }
}

// Serving, one BF16 pass over every chunk.  ANCH = false (problems without
// anchor tables): every query with the plain estimate.  ANCH = true: the
// queries of the list `sorted` (scnt entries, sorted by a slot), in tiles of
// 64 taken relative to the slot of the tile's first entry -- the error bound
// then scales with the distances to a nearby centroid instead of the norms,
// as in the filtered iterations.  A query whose decision is certain gets its
// label; any other goes to the list unc (ucnt entries), with its provisional
// best slot in ubest when given.
template <int KS, int DEPTH, bool ANCH>
__device__ __forceinline__ void b_serve(const ProbDev &P, const float *__restrict__ Q, long long nq,
                                        int *__restrict__ labels, const int2 *__restrict__ sorted,
                                        const unsigned long long *__restrict__ scnt, int *__restrict__ unc,
                                        int *__restrict__ ubest, unsigned long long *__restrict__ ucnt,
                                        const int bid_, const int nblk_)
{
    __shared__ BlockLds<KS> L;
    const int lane = lane_id(), pt = lane & 15, quad = lane >> 4, wv = threadIdx.x / WAVE;
    const Eta3 ek = mfma_eta3_coef(P.ldb);
    for (int i = threadIdx.x; i < P.g; i += blockDim.x) {   // every group, in order
        Visit &d = L.vis[i];
        d.g = i;
        d.s0 = P.gstart[i];
        d.ns = P.gsize[i];
        d.sgd = 0.f;
    }
    __syncthreads();
    ProbDev Pq = P;   // the query rows in place of the training points
    Pq.X = Q;
    const long long count = ANCH ? (long long)min(*scnt, (unsigned long long)nq) : nq;
    const long long ntiles = (count + 63) / 64;
    for (long long tl = bid_; tl < ntiles; tl += nblk_) {   // uniform per workgroup
        const long long e = tl * 64 + 16 * wv + pt;
        const bool in = e < count;
        long long q = e;
        Anchor anc = {-1, 0.f};
        if (ANCH) {
            q = in ? (long long)min(max(sorted[e].x, 0), (int)(nq - 1)) : 0;
            anc.a = clamp_slot(P, sorted[tl * 64].y);   // the tile's first entry is always listed
            anc.rt = (int)threadIdx.x < P.ldc ? P.c32[(size_t)anc.a * P.ldc + threadIdx.x] : 0.f;
            if ((int)threadIdx.x < 32 * KS) L.ar[threadIdx.x] = anc.rt;
            __syncthreads();
        }
        float v[KS][8];
        load_rows16<KS>(Pq, in ? (int)q : 0, in, v);
        float xnp;
        if (ANCH) {
            // x~ = fl(x - c_a) and its squared norm (FP64, rounded once)
            double sq = 0.0;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const float4 r0 = *(const float4 *)&L.ar[32 * ks + 8 * quad];
                const float4 r1 = *(const float4 *)&L.ar[32 * ks + 8 * quad + 4];
                const float rr[8] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const float xv = v[ks][j] - rr[j];
                    v[ks][j] = xv;
                    sq = fma((double)xv, (double)xv, sq);
                }
            }
            sq += __shfl_xor(sq, 16);
            sq += __shfl_xor(sq, 32);
            xnp = (float)sq;
        } else {
            xnp = norm_rows16<KS>(v);
        }
        PtFrag<KS> b;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) split8(v[ks], b.h[ks], b.l[ks]);
        const unsigned inm = (unsigned)__ballot(in) & 0xFFFFu;   // this wave's queries
        const float2 eA = mfma_eta3_pt(ek, mfma_eta3_a(xnp));
        RunB r;
        runb_init(r);
        float gmin = KP_INF;
        auto note = [&](int, unsigned, int, bool) {};
        auto fold1 = [&](int g, unsigned m, int slot0, bool first, float, const Key3 &kk) {
            const float l1 = key_value(kk.k1), l2 = key_value(kk.k2);
            const float gprev = first ? KP_INF : gmin;
            gmin = fminf(gprev, l1);
            runb_fold(r, (m >> pt) & 1u, l1, kk.u1, slot0 + (int)(kk.k1 & 15u), l2, g, gprev, false);
        };
        auto fold4 = [&](Key3 p0, Key3 p1, Key3 p2, Key3 p3, ChunkMeta m0, ChunkMeta m1, ChunkMeta m2, ChunkMeta m3,
                         int n) {
            const Key3 kk = key3_scatter4(p0, p1, p2, p3);
            const ChunkMeta mq = meta_of(quad, m0, m1, m2, m3);
            const bool mine = quad < n && ((mq.m >> pt) & 1u);
            runb_fold(r, mine, key_value(kk.k1), kk.u1, mq.slot0 + (int)(kk.k1 & 15u), key_value(kk.k2), mq.g,
                      KP_INF, false);
        };
        auto skip = [&]() {};
        auto src = [&](int k, int &g, unsigned &m, int &s0, int &ns, float &sgd) {
            g = k;
            m = inm;
            s0 = uni(L.vis[k].s0);
            ns = uni(L.vis[k].ns);
            sgd = uni(L.vis[k].sgd);
        };
        if (KS >= 4 && P.maxgs <= CHUNK) {   // as in the distance kernel
            block_visits<KS, DEPTH, true>(P, L, P.g, src, b, xnp, eA, anc, note, fold1, fold4, skip);
            r = runb_allreduce(r);
        } else {
            block_visits<KS, DEPTH, false>(P, L, P.g, src, b, xnp, eA, anc, note, fold1, fold4, skip);
        }
        bool amb = false;
        if (in && quad == 0) {
            // certain iff the best row's upper bound is below every other
            // row's lower bound
            const float Ub = root_hi(r.bu), Ls = root_lo(r.sec);
            if (Ub < Ls && r.bs >= 0) labels[q] = P.perm[clamp_slot(P, r.bs)];
            else amb = true;
        }
        const long long ea = wave_append(ucnt, amb);
        if (ea >= 0) {
            unc[ea] = (int)q;
            if (ubest) ubest[ea] = r.bs;
        }
    }
}
template <int KS, int DEPTH, bool ANCH>
__global__ __launch_bounds__(256) void k_serve(ProbDev P, const float *Q, long long nq, int *labels,
                                               const int2 *sorted, const unsigned long long *scnt, int *unc,
                                               int *ubest, unsigned long long *ucnt)
{
    b_serve<KS, DEPTH, ANCH>(P, Q, nq, labels, sorted, scnt, unc, ubest, ucnt, (int)blockIdx.x, (int)gridDim.x);
}

// Counting sort of listed queries by slot: the histogram, then (after
// k_scan) every entry placed at its slot's cursor.  Entry e is query unc[e]
// with slot ubest[e], or (unc == nullptr) query e itself.  Each workgroup
// takes a contiguous range of entries and counts it in LDS first (at most
// ANCHOR_MAX_SLOTS slots), so that the global counters take one atomic per
// (workgroup, slot) instead of one per entry: every query of the first
// anchored pass falls on one of only g medoid slots.
constexpr int SV_BLOCKS = 256;
__global__ __launch_bounds__(1024) void k_sv_hist(ProbDev P, const int *__restrict__ ubest,
                                                  const unsigned long long *__restrict__ ucnt, long long nq,
                                                  int *__restrict__ hist)
{
    __shared__ int h[ANCHOR_MAX_SLOTS];
    const long long cnt = (long long)min(*ucnt, (unsigned long long)nq);
    const long long per = (cnt + gridDim.x - 1) / gridDim.x;
    const long long e0 = (long long)blockIdx.x * per, e1 = min(cnt, e0 + per);
    const int kg = min(P.kg, (int)ANCHOR_MAX_SLOTS);
    for (int i = threadIdx.x; i < kg; i += blockDim.x) h[i] = 0;
    __syncthreads();
    for (long long e = e0 + threadIdx.x; e < e1; e += blockDim.x) atomicAdd(&h[min(clamp_slot(P, ubest[e]), kg - 1)], 1);
    __syncthreads();
    for (int i = threadIdx.x; i < kg; i += blockDim.x)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}
__global__ __launch_bounds__(1024) void k_sv_scatter(ProbDev P, const int *__restrict__ unc,
                                                     const int *__restrict__ ubest,
                                                     const unsigned long long *__restrict__ ucnt, long long nq,
                                                     int *__restrict__ cursor, int2 *__restrict__ sorted)
{
    __shared__ int h[ANCHOR_MAX_SLOTS];   // the range's count per slot, then its next place
    const long long cnt = (long long)min(*ucnt, (unsigned long long)nq);
    const long long per = (cnt + gridDim.x - 1) / gridDim.x;
    const long long e0 = (long long)blockIdx.x * per, e1 = min(cnt, e0 + per);
    const int kg = min(P.kg, (int)ANCHOR_MAX_SLOTS);
    for (int i = threadIdx.x; i < kg; i += blockDim.x) h[i] = 0;
    __syncthreads();
    for (long long e = e0 + threadIdx.x; e < e1; e += blockDim.x) atomicAdd(&h[min(clamp_slot(P, ubest[e]), kg - 1)], 1);
    __syncthreads();
    // this range's places: one reservation per slot it holds
    for (int i = threadIdx.x; i < kg; i += blockDim.x)
        if (h[i]) h[i] = atomicAdd(&cursor[i], h[i]);
    __syncthreads();
    for (long long e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        const int sl = min(clamp_slot(P, ubest[e]), kg - 1);
        const int pos = atomicAdd(&h[sl], 1);
        sorted[min(max(pos, 0), (int)(cnt - 1))] = make_int2(unc ? unc[e] : (int)e, sl);
    }
}

// FP32 direct form over every centroid, eight lanes per query (as the
// recheck), for the listed queries (unc != nullptr) or for all of them.
// Lowest original index on exact ties.
template <int NV>
__global__ __launch_bounds__(256) void k_serve_fp32(ProbDev P, const float *__restrict__ Q, long long nq,
                                                    const int *__restrict__ unc,
                                                    const unsigned long long *__restrict__ ucnt,
                                                    int *__restrict__ labels)
{
    const int lane = lane_id();
    const int t = lane & (RT - 1);
    const int team = threadIdx.x / RT;
    const long long cnt = unc ? (long long)min(*ucnt, (unsigned long long)nq) : nq;
    const long long nteams = (long long)gridDim.x * (blockDim.x / RT);
    const long long trips = (cnt + nteams - 1) / nteams;   // the same for every lane of the grid
    for (long long it = 0; it < trips; ++it) {
        const long long e = it * nteams + (long long)blockIdx.x * (blockDim.x / RT) + team;
        const bool live = e < cnt;
        if (__ballot(live) == 0ull) continue;
        const long long q = live ? (unc ? (long long)min(max(unc[e], 0), (int)(nq - 1)) : e) : 0;
        float4 x[NV];
        const float *xrow = Q + (size_t)q * P.d;
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const int i = 4 * t + 32 * j;
            float v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = (live && i + u < P.d) ? xrow[i + u] : 0.f;
            x[j] = make_float4(v[0], v[1], v[2], v[3]);
        }
        float bd = KP_INF;
        int bo = 0x7FFFFFFF;
        constexpr int BATCH = NV <= 4 ? 4 : 2;   // rows in flight together
        for (int s0 = 0; s0 < P.kg; s0 += BATCH) {
            float4 c4[BATCH][NV];
#pragma unroll
            for (int u = 0; u < BATCH; ++u)
                team_load<NV>(c4[u], P.c32 + (size_t)min(s0 + u, P.kg - 1) * P.ldc, P.ldc, t);
#pragma unroll
            for (int u = 0; u < BATCH; ++u) {
                const float dv = team_dist<NV>(x, c4[u]);
                const int o = s0 + u < P.kg ? P.perm[s0 + u] : -1;   // -1: padding slot
                if (o >= 0 && (dv < bd || (dv == bd && o < bo))) {
                    bd = dv;
                    bo = o;
                }
            }
        }
        if (live && t == 0) labels[q] = bo;
    }
}

// The listed queries in FP32 direct form over every centroid, a whole wave
// per query: its eight teams of eight lanes take interleaved runs of slots
// and combine their minima at the end (the list is short, so a query's
// latency, not the count, sets the time).  Lowest original index on exact
// ties.
template <int NV>
__global__ __launch_bounds__(256) void k_serve_fp32_list(ProbDev P, const float *__restrict__ Q, long long nq,
                                                         const int *__restrict__ unc,
                                                         const unsigned long long *__restrict__ ucnt,
                                                         int *__restrict__ labels)
{
    const int lane = lane_id();
    const int t = lane & (RT - 1), tw = lane / RT;   // lane in its team, team in the wave
    const long long cnt = (long long)min(*ucnt, (unsigned long long)nq);
    const long long nwaves = (long long)gridDim.x * (blockDim.x / WAVE);
    const long long wid = (long long)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    for (long long e = wid; e < cnt; e += nwaves) {   // uniform per wave
        const long long q = (long long)min(max(unc[e], 0), (int)(nq - 1));
        float4 x[NV];
        const float *xrow = Q + (size_t)q * P.d;
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const int i = 4 * t + 32 * j;
            float v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = i + u < P.d ? xrow[i + u] : 0.f;
            x[j] = make_float4(v[0], v[1], v[2], v[3]);
        }
        float bd = KP_INF;
        int bo = 0x7FFFFFFF;
        constexpr int BATCH = NV <= 4 ? 4 : 2;   // rows in flight per team
        for (int s0 = tw * BATCH; s0 < P.kg; s0 += (WAVE / RT) * BATCH) {
            float4 c4[BATCH][NV];
#pragma unroll
            for (int u = 0; u < BATCH; ++u)
                team_load<NV>(c4[u], P.c32 + (size_t)min(s0 + u, P.kg - 1) * P.ldc, P.ldc, t);
#pragma unroll
            for (int u = 0; u < BATCH; ++u) {
                const float dv = team_dist<NV>(x, c4[u]);
                const int o = s0 + u < P.kg ? P.perm[s0 + u] : -1;   // -1: padding slot
                if (o >= 0 && (dv < bd || (dv == bd && o < bo))) {
                    bd = dv;
                    bo = o;
                }
            }
        }
#pragma unroll
        for (int o = RT; o < WAVE; o <<= 1) {
            const float ob = __shfl_xor(bd, o);
            const int oo = __shfl_xor(bo, o);
            if (ob < bd || (ob == bd && oo < bo)) {
                bd = ob;
                bo = oo;
            }
        }
        if (lane == 0) labels[q] = bo;
    }
}

// ============================================================ diagnostics
// The estimates the distance kernels decide on, and their bounds, for query
// rows against every centroid: the same point split, chunk staging, matrix
// products, estimate and per-row bound as the assignment, one chunk at a
// time (no pipelining), every value written out instead of reduced (the
// kernels form L = v - e and U = v + e from them).  With
// an anchor slot (>= 0) every query is taken relative to that centroid, as
// the filtered iterations take a tile's points relative to its anchor.
template <int KS>
__global__ __launch_bounds__(256) void k_probe(ProbDev P, const float *__restrict__ Q, long long nq, int anchor,
                                               float *__restrict__ est, float *__restrict__ eta)
{
    __shared__ ChunkStage<KS> S;
    __shared__ float ar[32 * KS];
    const int lane = lane_id(), pt = lane & 15, quad = lane >> 4, wv = threadIdx.x / WAVE;
    const Eta3 ek = mfma_eta3_coef(P.ldb);
    const int t = threadIdx.x;
    const Anchor anc = {anchor, (anchor >= 0 && t < P.ldc) ? P.c32[(size_t)anchor * P.ldc + t] : 0.f};
    if (t < 32 * KS) ar[t] = anc.rt;
    __syncthreads();
    ProbDev Pq = P;
    Pq.X = Q;
    const long long ntiles = (nq + 63) / 64;
    for (long long tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {   // uniform per workgroup
        const long long q = tl * 64 + 16 * wv + pt;
        const bool in = q < nq;
        float v[KS][8];
        load_rows16<KS>(Pq, in ? (int)q : 0, in, v);
        float xnp;
        if (anchor >= 0) {
            double sq = 0.0;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    v[ks][j] -= ar[32 * ks + 8 * quad + j];
                    sq = fma((double)v[ks][j], (double)v[ks][j], sq);
                }
            sq += __shfl_xor(sq, 16);
            sq += __shfl_xor(sq, 32);
            xnp = (float)sq;
        } else {
            xnp = norm_rows16<KS>(v);
        }
        PtFrag<KS> b;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) split8(v[ks], b.h[ks], b.l[ks]);
        const float2 eA = mfma_eta3_pt(ek, mfma_eta3_a(xnp));
        for (int g = 0; g < P.g; ++g) {
            const int s0 = P.gstart[g], ns = P.gsize[g];
            for (int c0 = 0; c0 < ns; c0 += CHUNK) {
                StageRegs<KS> R;
                stage_load<KS>(P, s0 + c0, R, anc);
                __syncthreads();   // the previous chunk's reads are done
                stage_store<KS>(S, R, anc, P.ldc);
                __syncthreads();
                f32x4 hh, lo;
                chunk_acc<KS>(S, b, hh, lo);
                float ev[4], ee[4];
                chunk_est(hh, lo, S.cn[quad], xnp, ev);
                chunk_eta(eA, S.wt, S.cn[4 + quad], ee);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int off = c0 + 4 * quad + r;   // slot offset in the group
                    const int orig = off < ns ? P.perm[s0 + off] : -1;
                    if (in && orig >= 0) {
                        est[(size_t)q * P.k + orig] = ev[r];
                        eta[(size_t)q * P.k + orig] = ee[r];
                    }
                }
            }
        }
    }
}

// Bounds of listed points brought to the current centroids (offset form
// undone with the drift sums rounded the way the filters round them).
__global__ void k_bounds(ProbDev P, const int *__restrict__ idx, long long np, float *__restrict__ ub,
                         float *__restrict__ lbp, float *__restrict__ lb)
{
    const float sdu = P.Sdud[0], lsc = P.lbsc[0];
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < np;
         i += (long long)gridDim.x * blockDim.x) {
        const int pid = clamp_pid(P, idx[i]);
        const PointState s = P.st[pid];
        const int a = clamp_slot(P, s.a);
        ub[i] = ub_now(s.u, P.Scu[a]);
        lbp[i] = lb_now(s.p, sdu);
        for (int q = 0; q < P.g; ++q) {
            const size_t o = (size_t)pid * P.gs + q;
            const float v = (P.prec && P.lb16) ? lb16_dec(P.lbh[o], lsc) : P.lb[o];
            lb[(size_t)i * P.g + q] = lb_now(v, P.Sgu[q]);
        }
    }
}

__global__ void k_groups_out(ProbDev P, int *out)
{
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < P.kg; s += gridDim.x * blockDim.x) {
        const int o = P.perm[s];
        if (o >= 0) out[o] = P.slot_group[s];
    }
}

// ================================================================ outputs
__global__ void k_labels(ProbDev P, int *out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P.n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = P.perm[clamp_slot(P, P.st[i].a)];
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
template <bool LB16>
static void launch_recheck(const ProbDev &P, hipStream_t s, int blocks)
{
    if (P.ldc <= 32) hipLaunchKernelGGL((k_recheck<1, LB16>), dim3(blocks), dim3(256), 0, s, P);
    else if (P.ldc <= 64) hipLaunchKernelGGL((k_recheck<2, LB16>), dim3(blocks), dim3(256), 0, s, P);
    else if (P.ldc <= 128) hipLaunchKernelGGL((k_recheck<4, LB16>), dim3(blocks), dim3(256), 0, s, P);
    else hipLaunchKernelGGL((k_recheck<8, LB16>), dim3(blocks), dim3(256), 0, s, P);
}

static void launch_atab(const ProbDev &P, hipStream_t s)
{
    if (!P.anch) return;
    const int T = (P.kg + AT_T - 1) / AT_T;
    hipLaunchKernelGGL(k_atab, dim3(T, T), dim3(256), 0, s, P);
}

hipError_t launch_prep(const ProbDev &P, hipStream_t s, const float *init_dev)
{
    if (P.prec) hipLaunchKernelGGL(k_prep, dim3(cap_grid((P.n + 15) / 16, 4096)), dim3(256), 0, s, P);
    hipLaunchKernelGGL(k_centroids<true>, dim3(cap_grid((P.kg + 3) / 4, 4096)), dim3(256), 0, s, P, init_dev);
    hipLaunchKernelGGL(k_drift, dim3(1), dim3(1024), 0, s, P, 1);
    launch_atab(P, s);
    return hipGetLastError();
}

// BF16 mode: one workgroup per 64 positions; KS = ldb / 32 in {1, 2, 3, 4, 6, 8};
// DEPTH = chunks in flight (1 or 3; 1 is the default).
template <bool DENSE, int DEPTH>
static void launch_blk64_ks(const ProbDev &P, hipStream_t s, int grid)
{
    switch (P.ldb / 32) {
    case 1: hipLaunchKernelGGL((k_blk64<1, DENSE, DEPTH>), dim3(grid), dim3(256), 0, s, P); break;
    case 2: hipLaunchKernelGGL((k_blk64<2, DENSE, DEPTH>), dim3(grid), dim3(256), 0, s, P); break;
    case 3: hipLaunchKernelGGL((k_blk64<3, DENSE, DEPTH>), dim3(grid), dim3(256), 0, s, P); break;
    case 4: hipLaunchKernelGGL((k_blk64<4, DENSE, DEPTH>), dim3(grid), dim3(256), 0, s, P); break;
    case 6: hipLaunchKernelGGL((k_blk64<6, DENSE, DEPTH>), dim3(grid), dim3(256), 0, s, P); break;
    case 8: hipLaunchKernelGGL((k_blk64<8, DENSE, DEPTH>), dim3(grid), dim3(256), 0, s, P); break;
    default: break;   // excluded when the plan is made
    }
}
static void launch_blk64(const ProbDev &P, hipStream_t s, const LaunchCfg &cfg, bool dense)
{
    const int grid = cap_grid((P.n + 63) / 64, cfg.grid_cap);
    // the dense pass (every chunk for every tile) keeps three chunks in
    // flight; the filtered pass takes the tuned depth
    if (dense) launch_blk64_ks<true, 3>(P, s, grid);
    else if (cfg.depth == 1) launch_blk64_ks<false, 1>(P, s, grid);
    else launch_blk64_ks<false, 3>(P, s, grid);
}

static void launch_dense(const ProbDev &P, hipStream_t s, const LaunchCfg &cfg)
{
    const int threads = 64 * cfg.waves;
    const int grid = cap_grid(((P.n + 63) / 64 + cfg.waves - 1) / cfg.waves, cfg.grid_cap);
    if (P.prec == 0) {
        const int dm = P.ldc;
        if (dm <= 8) hipLaunchKernelGGL(k_dense_f32<8>, dim3(grid), dim3(threads), 0, s, P);
        else if (dm <= 16) hipLaunchKernelGGL(k_dense_f32<16>, dim3(grid), dim3(threads), 0, s, P);
        else if (dm <= 32) hipLaunchKernelGGL(k_dense_f32<32>, dim3(grid), dim3(threads), 0, s, P);
        else if (dm <= 64) hipLaunchKernelGGL(k_dense_f32<64>, dim3(grid), dim3(threads), 0, s, P);
        else hipLaunchKernelGGL(k_dense_f32<128>, dim3(grid), dim3(threads), 0, s, P);
    } else {
        launch_blk64(P, s, cfg, true);
    }
}

static void launch_survivors(const ProbDev &P, hipStream_t s, const LaunchCfg &cfg)
{
    const int threads = 64 * cfg.waves;
    const int grid = cap_grid(((P.n + 63) / 64 + cfg.waves - 1) / cfg.waves, cfg.grid_cap);
    const int gt_grid = cap_grid(((P.n + 63) / 64 + GT_WAVES - 1) / GT_WAVES, cfg.grid_cap);
    if (P.prec == 0) {
        hipLaunchKernelGGL(k_group_test, dim3(gt_grid), dim3(WAVE * GT_WAVES), 0, s, P);
        const int dm = P.ldc;
        if (dm <= 8) hipLaunchKernelGGL(k_tile_f32<8>, dim3(grid), dim3(threads), 0, s, P);
        else if (dm <= 16) hipLaunchKernelGGL(k_tile_f32<16>, dim3(grid), dim3(threads), 0, s, P);
        else if (dm <= 32) hipLaunchKernelGGL(k_tile_f32<32>, dim3(grid), dim3(threads), 0, s, P);
        else if (dm <= 64) hipLaunchKernelGGL(k_tile_f32<64>, dim3(grid), dim3(threads), 0, s, P);
        else hipLaunchKernelGGL(k_tile_f32<128>, dim3(grid), dim3(threads), 0, s, P);
    } else {
        launch_blk64(P, s, cfg, false);
    }
}

// FP64 accumulators per lane of the wave-per-row sums: ceil(d / 64), rounded
// up to 8 or 16 above 4.
static int dch_class_of(int d)
{
    const int c = (d + 63) / 64;
    return c <= 4 ? c : (c <= 8 ? 8 : 16);
}

// Deterministic mode: the scan of a (key, block) table of nkeys keys.
static void launch_ss_scan(const ProbDev &P, hipStream_t s, long long nkeys)
{
    const long long L = nkeys * SS_NB;
    hipLaunchKernelGGL(k_ss_scan_part, dim3(SS_SCAN_BLOCKS), dim3(256), 0, s, (const int *)P.hist2, L, P.spart);
    hipLaunchKernelGGL(k_ss_scan_top, dim3(1), dim3(1024), 0, s, P.spart);
    hipLaunchKernelGGL(k_ss_scan_fin, dim3(SS_SCAN_BLOCKS), dim3(256), 0, s, P.hist2, L, (const int *)P.spart);
}
static void launch_fill0(int *a, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill0, dim3(cap_grid((n + 255) / 256, 4096)), dim3(256), 0, s, a, n);
}
// Deterministic update: all points sorted by (slot, index), then the
// fixed-order sums.
template <int DCH>
static void launch_dsum(const ProbDev &P, hipStream_t s, int grid)
{
    hipLaunchKernelGGL(k_dsum_piece<DCH>, dim3(grid), dim3(256), 0, s, P);
    hipLaunchKernelGGL(k_dsum_fix<DCH>, dim3(cap_grid((P.kg + 3) / 4, 4096)), dim3(256), 0, s, P);
}
static void launch_update_det(const ProbDev &P, hipStream_t s, const LaunchCfg &cfg)
{
    launch_fill0(P.hist2, (long long)P.kg * SS_NB, s);
    hipLaunchKernelGGL(k_ss_hist_pts, dim3(SS_NB), dim3(64), 0, s, P);
    launch_ss_scan(P, s, P.kg);
    hipLaunchKernelGGL(k_ss_scatter_pts, dim3(SS_NB), dim3(64), 0, s, P);
    const int grid = cap_grid(((P.n + DS_PIECE - 1) / DS_PIECE + 3) / 4, cfg.grid_cap);
    switch (dch_class_of(P.d)) {
    case 1: launch_dsum<1>(P, s, grid); break;
    case 2: launch_dsum<2>(P, s, grid); break;
    case 3: launch_dsum<3>(P, s, grid); break;
    case 4: launch_dsum<4>(P, s, grid); break;
    case 8: launch_dsum<8>(P, s, grid); break;
    default: launch_dsum<16>(P, s, grid); break;
    }
}

static void launch_update(const ProbDev &P, hipStream_t s, const LaunchCfg &cfg)
{
    if (P.det) {
        launch_update_det(P, s, cfg);
        return;
    }
    const int ublocks = cap_grid((2 * P.n + 255) / 256, cfg.grid_cap);
    hipLaunchKernelGGL(k_hist, dim3(ublocks), dim3(256), 0, s, P);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, (const int *)P.hist, P.cursor, P.kg);
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
    launch_atab(P, s);
}

const char *stage_name(Stage st)
{
    static const char *names[ST_COUNT] = {"begin", "bound_filter", "l1_sort", "assign_dense", "group_filter",
                                          "assign", "recheck", "update", "centroids"};
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
        out[n++] = ST_SORT;
        if (P.prec) out[n++] = ST_GFILTER;
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
        hipLaunchKernelGGL(k_begin, dim3(cap_grid(((long long)P.nk1 + 256) / 256, 1024)), dim3(256), 0, s, P, dense ? 1 : 0);
        break;
    case ST_FILTER: {
        const int grid = cap_grid((P.n + BF_CHUNK - 1) / BF_CHUNK, cfg.grid_cap);
        if (P.g <= GMAX_BF16)   // returns at once unless the row test is on
            hipLaunchKernelGGL(k_row_pre, dim3(cap_grid((P.n + 255) / 256, std::min(cfg.grid_cap, 2048))), dim3(256), 0,
                               s, P);
        if (P.det) {
            hipLaunchKernelGGL(k_bf_count, dim3(grid), dim3(256), 0, s, P);
            hipLaunchKernelGGL(k_bf_scan, dim3(1), dim3(1024), 0, s, P, (int)((P.n + BF_CHUNK - 1) / BF_CHUNK));
        }
        hipLaunchKernelGGL(k_bound_filter, dim3(grid), dim3(256), 0, s, P);
        break;
    }
    case ST_SORT: {
        if (P.det) {
            launch_fill0(P.hist2, (long long)P.nk1 * SS_NB, s);
            hipLaunchKernelGGL(k_ss_hist_l1, dim3(SS_NB), dim3(64), 0, s, P);
            launch_ss_scan(P, s, P.nk1);
            hipLaunchKernelGGL(k_ss_scatter_l1, dim3(SS_NB), dim3(64), 0, s, P);
            break;
        }
        const int blocks = cap_grid((P.n + 16383) / 16384, 1024);
        hipLaunchKernelGGL(k_key_hist, dim3(blocks), dim3(256), 0, s, P);
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, (const int *)P.hist1, P.cursor1, P.nk1);
        hipLaunchKernelGGL(k_l1_scatter, dim3(blocks), dim3(256), 0, s, P);
        break;
    }
    case ST_ASSIGN_DENSE: launch_dense(P, s, cfg); break;
    case ST_GFILTER:
        if (P.lb16) hipLaunchKernelGGL(k_gfilter<true>, dim3(cap_grid(((P.n + 15) / 16 + 3) / 4, cfg.grid_cap)), dim3(256), 0, s, P);
        else hipLaunchKernelGGL(k_gfilter<false>, dim3(cap_grid(((P.n + 15) / 16 + 3) / 4, cfg.grid_cap)), dim3(256), 0, s, P);
        break;
    case ST_ASSIGN: launch_survivors(P, s, cfg); break;
    case ST_RECHECK: {
        const int blocks = cap_grid((P.n + 31) / 32, cfg.grid_cap);
        if (P.lb16) launch_recheck<true>(P, s, blocks);
        else launch_recheck<false>(P, s, blocks);
        break;
    }
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
        const hipError_t e = launch_stage(P, s, sts[i], dense, cfg);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ------------------------------------------------------------- batches
static int dmax_class(int ldc) { return ldc <= 8 ? 0 : ldc <= 16 ? 1 : ldc <= 32 ? 2 : ldc <= 64 ? 3 : 4; }
static int ks_class(int ldb)
{
    switch (ldb / 32) {
    case 1: return 0;
    case 2: return 1;
    case 3: return 2;
    case 4: return 3;
    case 6: return 4;
    default: return 5;
    }
}
static int nv_class(int ldc) { return ldc <= 32 ? 0 : ldc <= 64 ? 1 : ldc <= 128 ? 2 : 3; }
static int dch_class(int d)
{
    const int c = (d + 63) / 64;
    return c <= 4 ? c - 1 : c <= 8 ? 4 : 5;
}

// Blocks of problem P in table id (the shapes of the single-problem launches
// above, with `cap` for the grid-stride kernels).
static int tab_blocks(int id, const ProbDev &P, const LaunchCfg &cfg, int cap)
{
    const long long n = P.n;
    const bool f32 = P.prec == 0;
    if (id >= TB_DENSE_F32 && id < TB_TILE_F32)
        return f32 && dmax_class(P.ldc) == id - TB_DENSE_F32 ? cap_grid(((n + 63) / 64 + cfg.waves - 1) / cfg.waves, cap)
                                                              : 0;
    if (id >= TB_TILE_F32 && id < TB_BLK64)
        return f32 && dmax_class(P.ldc) == id - TB_TILE_F32 ? cap_grid(((n + 63) / 64 + cfg.waves - 1) / cfg.waves, cap)
                                                             : 0;
    if (id >= TB_BLK64 && id < TB_RECHECK)
        return !f32 && ks_class(P.ldb) == id - TB_BLK64 ? cap_grid((n + 63) / 64, cap) : 0;
    if (id >= TB_RECHECK && id < TB_SEGSUM)
        return !f32 && nv_class(P.ldc) == id - TB_RECHECK ? cap_grid((n + 31) / 32, cap) : 0;
    if (id >= TB_SEGSUM && id < TB_COUNT)
        return dch_class(P.d) == id - TB_SEGSUM ? cap_grid((2 * n + 255) / 256, cap) : 0;
    switch (id) {
    case TB_BEGIN: return cap_grid(((long long)P.nk1 + 256) / 256, 1024);
    case TB_FILTER: return cap_grid((n + 4095) / 4096, cap);
    case TB_ROWPRE: return P.g <= GMAX_BF16 ? cap_grid((n + 255) / 256, std::min(cap, 2048)) : 0;
    case TB_SORT: return cap_grid((n + 16383) / 16384, 1024);
    case TB_ONE: return 1;
    case TB_CENT: return cap_grid((P.kg + 3) / 4, 4096);
    case TB_GT: return f32 ? cap_grid(((n + 63) / 64 + GT_WAVES - 1) / GT_WAVES, cap) : 0;
    case TB_GF: return f32 ? 0 : cap_grid(((n + 15) / 16 + 3) / 4, cap);
    case TB_HIST: return cap_grid((2 * n + 255) / 256, cap);
    case TB_SCATTER: return cap_grid((2 * n + 4095) / 4096, 1024);
    case TB_ATAB: {
        const int T = (P.kg + AT_T - 1) / AT_T;
        return P.anch ? T * T : 0;
    }
    default: return 0;
    }
}

void build_tables(Batch &B, const std::vector<ProbDev> &hp, const LaunchCfg &cfg)
{
    const int count = (int)hp.size();
    B.count = count;
    B.htabs.assign((size_t)TB_COUNT * (count + 1), 0);
    double ntot = 0.0;
    for (const ProbDev &P : hp) ntot += (double)P.n;
    for (int id = 0; id < TB_COUNT; ++id) {
        int *t = &B.htabs[(size_t)id * (count + 1)];
        long long acc = 0;
        for (int i = 0; i < count; ++i) {
            // grid-stride kernels: four times the single-problem cap, shared in proportion to N
            const int cap = count == 1 ? cfg.grid_cap
                                       : (int)std::max(8.0, std::ceil(4.0 * cfg.grid_cap * (double)hp[i].n / ntot));
            t[i] = (int)acc;
            acc += tab_blocks(id, hp[i], cfg, cap);
        }
        t[count] = (int)acc;
    }
}

int batch_stages(const std::vector<ProbDev> &hp, bool dense, Stage out[ST_COUNT])
{
    bool any_bf16 = false;
    for (const ProbDev &P : hp) any_bf16 |= P.prec != 0;
    int n = 0;
    out[n++] = ST_BEGIN;
    if (dense) {
        out[n++] = ST_ASSIGN_DENSE;
    } else {
        out[n++] = ST_FILTER;
        out[n++] = ST_SORT;
        if (any_bf16) out[n++] = ST_GFILTER;
        out[n++] = ST_ASSIGN;
    }
    if (any_bf16) out[n++] = ST_RECHECK;
    out[n++] = ST_UPDATE;
    out[n++] = ST_CENTROIDS;
    return n;
}

#define KB_LAUNCH(id, kern, threads, ...)                                                                   \
    do {                                                                                                    \
        const int tot_ = B.total(id);                                                                       \
        if (tot_ > 0) hipLaunchKernelGGL(kern, dim3(tot_), dim3(threads), 0, s, B.probs, B.tab(id), B.count, \
                                         ##__VA_ARGS__);                                                    \
    } while (0)

template <bool DENSE, int DEPTH>
static void batch_blk64(const Batch &B, hipStream_t s)
{
    KB_LAUNCH(TB_BLK64 + 0, (kb_blk64<1, DENSE, DEPTH>), 256);
    KB_LAUNCH(TB_BLK64 + 1, (kb_blk64<2, DENSE, DEPTH>), 256);
    KB_LAUNCH(TB_BLK64 + 2, (kb_blk64<3, DENSE, DEPTH>), 256);
    KB_LAUNCH(TB_BLK64 + 3, (kb_blk64<4, DENSE, DEPTH>), 256);
    KB_LAUNCH(TB_BLK64 + 4, (kb_blk64<6, DENSE, DEPTH>), 256);
    KB_LAUNCH(TB_BLK64 + 5, (kb_blk64<8, DENSE, DEPTH>), 256);
}

hipError_t launch_stage_batch(const Batch &B, hipStream_t s, Stage st, bool dense, const LaunchCfg &cfg)
{
    const int wthreads = 64 * cfg.waves;
    switch (st) {
    case ST_BEGIN: KB_LAUNCH(TB_BEGIN, kb_begin, 256, dense ? 1 : 0); break;
    case ST_FILTER:
        KB_LAUNCH(TB_ROWPRE, kb_row_pre, 256);   // returns at once unless the problem's row test is on
        KB_LAUNCH(TB_FILTER, kb_bound_filter, 256);
        break;
    case ST_SORT:
        KB_LAUNCH(TB_SORT, kb_key_hist, 256);
        KB_LAUNCH(TB_ONE, kb_scan, 1024, 1);
        KB_LAUNCH(TB_SORT, kb_l1_scatter, 256);
        break;
    case ST_ASSIGN_DENSE:
        KB_LAUNCH(TB_DENSE_F32 + 0, kb_dense_f32<8>, wthreads);
        KB_LAUNCH(TB_DENSE_F32 + 1, kb_dense_f32<16>, wthreads);
        KB_LAUNCH(TB_DENSE_F32 + 2, kb_dense_f32<32>, wthreads);
        KB_LAUNCH(TB_DENSE_F32 + 3, kb_dense_f32<64>, wthreads);
        KB_LAUNCH(TB_DENSE_F32 + 4, kb_dense_f32<128>, wthreads);
        batch_blk64<true, 3>(B, s);   // the dense pass keeps three chunks in flight
        break;
    case ST_GFILTER:
        if (cfg.lb16) KB_LAUNCH(TB_GF, kb_gfilter<true>, 256);
        else KB_LAUNCH(TB_GF, kb_gfilter<false>, 256);
        break;
    case ST_ASSIGN:
        KB_LAUNCH(TB_GT, kb_group_test, WAVE * GT_WAVES);
        KB_LAUNCH(TB_TILE_F32 + 0, kb_tile_f32<8>, wthreads);
        KB_LAUNCH(TB_TILE_F32 + 1, kb_tile_f32<16>, wthreads);
        KB_LAUNCH(TB_TILE_F32 + 2, kb_tile_f32<32>, wthreads);
        KB_LAUNCH(TB_TILE_F32 + 3, kb_tile_f32<64>, wthreads);
        KB_LAUNCH(TB_TILE_F32 + 4, kb_tile_f32<128>, wthreads);
        if (cfg.depth == 1) batch_blk64<false, 1>(B, s);
        else batch_blk64<false, 3>(B, s);
        break;
    case ST_RECHECK:
        if (cfg.lb16) {
            KB_LAUNCH(TB_RECHECK + 0, (kb_recheck<1, true>), 256);
            KB_LAUNCH(TB_RECHECK + 1, (kb_recheck<2, true>), 256);
            KB_LAUNCH(TB_RECHECK + 2, (kb_recheck<4, true>), 256);
            KB_LAUNCH(TB_RECHECK + 3, (kb_recheck<8, true>), 256);
        } else {
            KB_LAUNCH(TB_RECHECK + 0, (kb_recheck<1, false>), 256);
            KB_LAUNCH(TB_RECHECK + 1, (kb_recheck<2, false>), 256);
            KB_LAUNCH(TB_RECHECK + 2, (kb_recheck<4, false>), 256);
            KB_LAUNCH(TB_RECHECK + 3, (kb_recheck<8, false>), 256);
        }
        break;
    case ST_UPDATE:
        KB_LAUNCH(TB_HIST, kb_hist, 256);
        KB_LAUNCH(TB_ONE, kb_scan, 1024, 0);
        KB_LAUNCH(TB_SCATTER, kb_scatter, 256);
        KB_LAUNCH(TB_SEGSUM + 0, kb_segsum<1>, 256);
        KB_LAUNCH(TB_SEGSUM + 1, kb_segsum<2>, 256);
        KB_LAUNCH(TB_SEGSUM + 2, kb_segsum<3>, 256);
        KB_LAUNCH(TB_SEGSUM + 3, kb_segsum<4>, 256);
        KB_LAUNCH(TB_SEGSUM + 4, kb_segsum<8>, 256);
        KB_LAUNCH(TB_SEGSUM + 5, kb_segsum<16>, 256);
        break;
    case ST_CENTROIDS:
        KB_LAUNCH(TB_CENT, kb_centroids<false>, 256, (const float *)nullptr);
        KB_LAUNCH(TB_ONE, kb_drift, 1024, 0);
        KB_LAUNCH(TB_ATAB, kb_atab, 256);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
#undef KB_LAUNCH

hipError_t launch_labels(const ProbDev &P, hipStream_t s, int *out)
{
    hipLaunchKernelGGL(k_labels, dim3(cap_grid((P.n + 255) / 256, 4096)), dim3(256), 0, s, P, out);
    return hipGetLastError();
}

// ------------------------------------------------ serving without allocation
// Scratch of kp_predict_noalloc, laid out as serve_scratch_bytes describes
// for NOALLOC_MAX_QUERIES queries with anchors (about 64 MiB: 16 bytes per
// query and the slot histogram).  Each device the library runs on holds its
// own copy until the process ends.  In host
// code the array's name is not a device address: its address on a device is
// taken once with hipGetSymbolAddress, with that device current, and kept.
static __device__ __align__(256) unsigned char scratch[serve_scratch_bytes(NOALLOC_MAX_QUERIES, true)];
constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

hipError_t noalloc_scratch_setup(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = ptr;
    return hipSuccess;
}

void *noalloc_scratch(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

hipError_t launch_serve(const ProbDev &P, hipStream_t s, const LaunchCfg &cfg, const float *Q, long long nq,
                        int *labels, void *scratch)
{
    // scratch layout: see serve_scratch_bytes
    char *base = (char *)scratch;
    auto *ucnt = (unsigned long long *)base;   // uncertain after the first and second pass; nq
    int *unc = (int *)(base + SERVE_HEADER);
    int *ubest = (int *)((char *)unc + serve_up((size_t)nq * 4));
    int2 *sorted = (int2 *)((char *)ubest + serve_up((size_t)nq * 4));
    int *hist = (int *)((char *)sorted + serve_up((size_t)nq * 8));
    int *cursor = hist + (ANCHOR_MAX_SLOTS + 1);
    const bool two = P.prec && P.anch;   // anchored passes
    const int nv = P.d <= 32 ? 1 : P.d <= 64 ? 2 : P.d <= 128 ? 4 : 8;
    const int grid2 = cap_grid((nq + 31) / 32, cfg.grid_cap);
    const unsigned long long *cnt_in = nullptr;
    const int *list = nullptr;
    if (P.prec) {
        hipLaunchKernelGGL(k_serve_begin, dim3(1), dim3(1), 0, s, ucnt, nq);
        const int grid = cap_grid((nq + 63) / 64, cfg.grid_cap);
#define KP_SERVE(KS, ANCH, SRT, SCNT, UB, CNT)                                                                  \
    hipLaunchKernelGGL((k_serve<KS, 1, ANCH>), dim3(grid), dim3(256), 0, s, P, Q, nq, labels, SRT, SCNT, unc, UB, CNT)
#define KP_SERVE_KS(ANCH, SRT, SCNT, UB, CNT)          \
    switch (P.ldb / 32) {                             \
    case 1: KP_SERVE(1, ANCH, SRT, SCNT, UB, CNT); break; \
    case 2: KP_SERVE(2, ANCH, SRT, SCNT, UB, CNT); break; \
    case 3: KP_SERVE(3, ANCH, SRT, SCNT, UB, CNT); break; \
    case 4: KP_SERVE(4, ANCH, SRT, SCNT, UB, CNT); break; \
    case 6: KP_SERVE(6, ANCH, SRT, SCNT, UB, CNT); break; \
    case 8: KP_SERVE(8, ANCH, SRT, SCNT, UB, CNT); break; \
    default: break; /* excluded when the plan is made */ \
    }
        if (two) {
            // every query anchored at its nearest chunk medoid, sorted by it
            hipLaunchKernelGGL(k_fill0, dim3(cap_grid((P.kg + 255) / 256, 64)), dim3(256), 0, s, hist, (long long)P.kg);
            switch (P.ldb / 32) {
            case 1: hipLaunchKernelGGL(k_serve_pre<1>, dim3(grid), dim3(256), 0, s, P, Q, nq, ubest); break;
            case 2: hipLaunchKernelGGL(k_serve_pre<2>, dim3(grid), dim3(256), 0, s, P, Q, nq, ubest); break;
            case 3: hipLaunchKernelGGL(k_serve_pre<3>, dim3(grid), dim3(256), 0, s, P, Q, nq, ubest); break;
            case 4: hipLaunchKernelGGL(k_serve_pre<4>, dim3(grid), dim3(256), 0, s, P, Q, nq, ubest); break;
            case 6: hipLaunchKernelGGL(k_serve_pre<6>, dim3(grid), dim3(256), 0, s, P, Q, nq, ubest); break;
            case 8: hipLaunchKernelGGL(k_serve_pre<8>, dim3(grid), dim3(256), 0, s, P, Q, nq, ubest); break;
            default: break;
            }
            hipLaunchKernelGGL(k_sv_hist, dim3(SV_BLOCKS), dim3(1024), 0, s, P, ubest, ucnt + 2, nq, hist);
            hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, hist, cursor, P.kg);
            hipLaunchKernelGGL(k_sv_scatter, dim3(SV_BLOCKS), dim3(1024), 0, s, P, (const int *)nullptr, ubest,
                               ucnt + 2, nq, cursor, sorted);
            // pass A: every query relative to its anchor; the uncertain ones
            // with their provisional best slot (overwriting the anchors,
            // whose entries are in `sorted` by then)
            KP_SERVE_KS(true, (const int2 *)sorted, (const unsigned long long *)(ucnt + 2), ubest, ucnt);
            // pass B: those, sorted by that slot, relative to it
            hipLaunchKernelGGL(k_fill0, dim3(cap_grid((P.kg + 255) / 256, 64)), dim3(256), 0, s, hist, (long long)P.kg);
            hipLaunchKernelGGL(k_sv_hist, dim3(SV_BLOCKS), dim3(1024), 0, s, P, ubest, ucnt, nq, hist);
            hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, hist, cursor, P.kg);
            hipLaunchKernelGGL(k_sv_scatter, dim3(SV_BLOCKS), dim3(1024), 0, s, P, unc, ubest, ucnt, nq, cursor, sorted);
            KP_SERVE_KS(true, (const int2 *)sorted, (const unsigned long long *)ucnt, (int *)nullptr, ucnt + 1);
            cnt_in = ucnt + 1;
        } else {
            // no anchor tables: one pass with the plain estimate
            KP_SERVE_KS(false, (const int2 *)nullptr, (const unsigned long long *)nullptr, (int *)nullptr, ucnt);
            cnt_in = ucnt;
        }
#undef KP_SERVE_KS
#undef KP_SERVE
        list = unc;
    }
    if (list) {   // the queries the BF16 passes left: a wave each
        const int gw = cap_grid((nq + 3) / 4, cfg.grid_cap);
        switch (nv) {
        case 1: hipLaunchKernelGGL(k_serve_fp32_list<1>, dim3(gw), dim3(256), 0, s, P, Q, nq, list, cnt_in, labels); break;
        case 2: hipLaunchKernelGGL(k_serve_fp32_list<2>, dim3(gw), dim3(256), 0, s, P, Q, nq, list, cnt_in, labels); break;
        case 4: hipLaunchKernelGGL(k_serve_fp32_list<4>, dim3(gw), dim3(256), 0, s, P, Q, nq, list, cnt_in, labels); break;
        default: hipLaunchKernelGGL(k_serve_fp32_list<8>, dim3(gw), dim3(256), 0, s, P, Q, nq, list, cnt_in, labels); break;
        }
        return hipGetLastError();
    }
    switch (nv) {
    case 1: hipLaunchKernelGGL(k_serve_fp32<1>, dim3(grid2), dim3(256), 0, s, P, Q, nq, list, cnt_in, labels); break;
    case 2: hipLaunchKernelGGL(k_serve_fp32<2>, dim3(grid2), dim3(256), 0, s, P, Q, nq, list, cnt_in, labels); break;
    case 4: hipLaunchKernelGGL(k_serve_fp32<4>, dim3(grid2), dim3(256), 0, s, P, Q, nq, list, cnt_in, labels); break;
    default: hipLaunchKernelGGL(k_serve_fp32<8>, dim3(grid2), dim3(256), 0, s, P, Q, nq, list, cnt_in, labels); break;
    }
    return hipGetLastError();
}

hipError_t launch_probe(const ProbDev &P, hipStream_t s, const float *Q, long long nq, int anchor, float *est,
                        float *eta)
{
    const int grid = cap_grid((nq + 63) / 64, 4096);
    switch (P.ldb / 32) {
    case 1: hipLaunchKernelGGL(k_probe<1>, dim3(grid), dim3(256), 0, s, P, Q, nq, anchor, est, eta); break;
    case 2: hipLaunchKernelGGL(k_probe<2>, dim3(grid), dim3(256), 0, s, P, Q, nq, anchor, est, eta); break;
    case 3: hipLaunchKernelGGL(k_probe<3>, dim3(grid), dim3(256), 0, s, P, Q, nq, anchor, est, eta); break;
    case 4: hipLaunchKernelGGL(k_probe<4>, dim3(grid), dim3(256), 0, s, P, Q, nq, anchor, est, eta); break;
    case 6: hipLaunchKernelGGL(k_probe<6>, dim3(grid), dim3(256), 0, s, P, Q, nq, anchor, est, eta); break;
    case 8: hipLaunchKernelGGL(k_probe<8>, dim3(grid), dim3(256), 0, s, P, Q, nq, anchor, est, eta); break;
    default: return hipErrorInvalidValue;   // excluded when the plan is made
    }
    return hipGetLastError();
}

hipError_t launch_bounds(const ProbDev &P, hipStream_t s, const int *idx, long long np, float *ub, float *lbp,
                         float *lb, int *groups)
{
    if (np > 0)
        hipLaunchKernelGGL(k_bounds, dim3(cap_grid((np + 255) / 256, 4096)), dim3(256), 0, s, P, idx, np, ub, lbp, lb);
    if (groups) hipLaunchKernelGGL(k_groups_out, dim3(cap_grid((P.kg + 255) / 256, 1024)), dim3(256), 0, s, P, groups);
    return hipGetLastError();
}

hipError_t launch_centroids_out(const ProbDev &P, hipStream_t s, float *c32, double *c64)
{
    hipLaunchKernelGGL(k_centroids_out, dim3(cap_grid(((long long)P.kg * P.d + 255) / 256, 4096)), dim3(256), 0,
                       s, P, c32, c64);
    return hipGetLastError();
}

}  // namespace kp
