// Device-side data layout and numeric helpers of the filtered K-means library.
//
// Layout in HBM (per problem, all carved from the caller's workspace):
//   X      n x d   FP32  caller's points, row-major, borrowed
//   xn     n       FP32  ||X_i||^2 (BF16 mode; the BF16 split of a point is
//                        formed on the fly in LDS, ldb = roundup(d, 32))
//   st     n       16 B  PointState: assigned slot and two bounds
//   lb     n x gs  group-level lower bounds: FP32, gs = roundup(g, 4) (FP32 mode);
//                 FP32 or FP16 codes in 128-byte rows (BF16 mode)
//   centroids in "slot" order: the members of group q occupy slots
//   gstart[q] .. gstart[q] + gsize[q] - 1 in ascending original index, and the
//   group is padded with empty slots to a multiple of 16 so that every
//   16-slot chunk of a MFMA tile belongs to one group.
//
// Bounds are stored in offset form against the cumulative drift of the
// centroids (FP64 sums, updated once per iteration):
//   Sc[j] = sum over updates of ||c_j(new) - c_j(old)||        (per slot)
//   Sg[q] = sum over updates of max_{j in q} drift              (per group)
//   Sd    = sum over updates of max_j drift                     (global)
// A point stores u = ub - Sc[a], p = lbp + Sd and v_q = lb_q + Sg[q] at the
// time the bound was computed; at any later iteration ub + (drift of c_a
// since then) = u + Sc[a], and similarly for the lower bounds.  This is the
// triangle inequality |d(x, c') - d(x, c)| <= ||c' - c|| accumulated over the
// iterations since the bound was last computed, without touching the point
// in between.  FP32 copies of the sums rounded up (evaluation) and down
// (storage) keep every bound valid under rounding.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kp {

constexpr int WAVE = 64;
constexpr int CHUNK = 16;             // centroid slots per MFMA tile / group padding
constexpr int STATS_CAP = 1024;       // per-iteration stats ring
constexpr int NCTR = 9;               // per-iteration counters
constexpr int HIST_LDS = 8192;        // largest slot count histogrammed in LDS
constexpr int L1_HIST = 16384;        // largest key count of the L1 order histogrammed in LDS
// Buckets of the nearest other group in the L1 order of a problem with n
// points, kg slots and g groups: as many as keep kg * buckets within the LDS
// histogram and about four tiles of 64 points per bucket, at most g + 1
// (1: order by slot only).
__host__ __device__ inline int l1_buckets(long long n, int kg, int g)
{
    if (kg <= 0) return 1;
    long long b = L1_HIST / kg;
    const long long fill = n / (256ll * kg);
    if (fill < b) b = fill;
    if (g + 1 < b) b = g + 1;
    return b < 1 ? 1 : (int)b;
}
constexpr int SINK_SLOTS = 1024;      // 64-byte slots taking the stores of lanes with nothing to write
constexpr int GMAX_BF16 = 1024;       // largest g of the BF16 mode (group tables kept in LDS)

// counters (unsigned long long) per problem
enum { CTR_L1 = 0, CTR_L3 = 1 /* rechecks */, CTR_MOVED = 2, CTR_PAIRS = 3, CTR_DIST = 4, CTR_DENSE = 5, CTR_VISITS = 6,
       CTR_MV = 7 /* entries of the moved list */,
       CTR_CLOSED = 8 /* points with every group closed, their own included */ };

struct __attribute__((aligned(16))) PointState {
    int a;        // slot of the assigned centroid
    float u;      // ub - Sc[a] (rounded up)
    float p;      // lbp + Sd (rounded down): lbp bounds min_{j != a} d(x, c_j)
    int ga;       // group of slot a
};

typedef __bf16 bf16x8 __attribute__((__vector_size__(8 * sizeof(__bf16))));
typedef float f32x4 __attribute__((__vector_size__(4 * sizeof(float))));

struct ProbDev {
    int64_t n;
    int d, k, g, kg;          // kg = number of slots (with padding)
    int ldc, ldb, gs;         // leading dims: c32 (roundup 4), bf16 (roundup 32), lb row
    int prec;                 // 0 fp32 direct, 1 bf16 + recheck
    int maxgs;                // largest group size (real members)
    int nk1;                  // keys of the L1 order: kg * buckets of the nearest other group (<= HIST_LDS), or kg
    const float *X;
    float *xn;
    PointState *st;
    float *lb;                // FP32 mode: lower bounds per (point, group), row stride gs
    uint16_t *lbh;            // BF16 mode with lb16: the same as FP16 codes (lb16_enc), row stride gs
    int lb16;                 // BF16 mode: 1 = bounds stored as FP16 codes, 0 = FP32
    float *lbsc;              // BF16 mode: [0] 2^e and [1] 2^-e of the FP16 codes, [2] bits of max ||x||^2
    float *c32;
    uint16_t *cb, *cbl;       // BF16 split of c32: cb = bf16(c), cbl = bf16(c - cb)
    float *cn;                // ||c32||^2 (BF16 mode; +inf for padding)
    double *c64, *sums, *delta;
    int *cnt;
    const int *perm;          // slot -> original index, -1 for padding
    const int *slot_group;    // slot -> group, -1 for padding
    const int *gstart, *gsize;
    double *Sc, *Sg, *Sd;     // cumulative drifts (kg, g, 1), FP64
    float *Scu, *Scd;         // FP32 copies of Sc rounded up / down
    float *Sgu, *Sgd;         // FP32 copies of Sg rounded up / down
    float *slk;               // per slot: its group's largest drift in the last update minus its own
                              // drift, rounded down (0 before the first update and for padding)
    int nch;                  // 16-slot chunks: kg / CHUNK (every group is padded to whole chunks)
    float *nrel;              // per slot j: ||fl(c_j - c_f)|| rounded up, f the first slot of j's chunk (0 for f)
    float2 *Wu;               // per chunk: (W, c W^2) of the estimate without an anchor, W >= ||c_f||
    int anch;                 // BF16 mode: filtered tiles take their estimates relative to an anchor centroid
    float *Qt;                // anch: kg x kg, ||c_j - c_a||^2 (row a, column j; FP64, rounded to nearest; +inf
                              // for padding j)
    float2 *Wa;               // anch: kg x nch, (W, c W^2) per (anchor a, chunk), W >= ||c_f - c_a||
    float *Sdud;              // [0] Sd rounded up, [1] Sd rounded down
    int4 *L1;                 // points failing the point-level filter (filter order): {point, slot, ub now, group field}
    int *L1s;                 // FP32 mode: the same ids sorted by assigned slot (and nearest other group, bucketed)
    int4 *L1x;                // per sorted entry: point, slot a, ub now (FP32 bits, rounded up), group of a
    int *L3;                  // positions of the points whose BF16 decision is uncertain
    float *minnc;             // per position: smallest bound of the closed groups (rounded down)
    int4 *tlist;              // per tile of sorted L1, g entries: the group filter's visit list
                              // (FP32: group, point mask lo, hi, 0; BF16: group, four 16-bit masks, 0)
    int *tcnt;                // entries used per tile
    float4 *ps4;              // per position: ub, min closed-group bound, U* of an uncertain point
    int *psf;                 // per position: bit 0 open (filter to distance kernel), bit 2 uncertain
    int *mv_pt, *mv_old, *mv_new;   // per position: point, old slot, new slot (-1: did not move)
    int *srt_pt, *srt_key;    // update entries sorted by centroid slot (sign in bit 31 of srt_pt)
    int *hist, *cursor;       // kg + 1: centroid update sort
    int *hist1, *cursor1;     // nk1 + 1: L1 sort
    unsigned long long *ctr;  // NCTR counters of the running iteration
    int *rowt;                // 1: the point-level filter tests whole bound rows this iteration (set by
                              // the previous iteration's drift step from its count of closed points)
    unsigned *rclosed;        // with rowt: bit i of word i / 32 set for point i when every group is closed
    long long *stats;         // STATS_CAP x 16
    int *iter;                // completed iterations
    float *sink;              // SINK_SLOTS x 16 floats, written and never read
    // deterministic mode (kp_tuning.deterministic): fixed-order lists and sums
    int det;                  // 1: the list of point-filter failures and the centroid sums in a fixed order
    int lf;                   // FP32 problems: 1 = the per-centroid local filter in the tile kernel
    int nb_l1, nb_slot;       // bits of the largest L1 key (nk1 - 1) and slot (kg - 1)
    int *dcnt, *doff;         // per chunk of BF_CHUNK points: failures, their first position in L1
    int *hist2;               // (key, block) counts of the stable counting sorts, then their cursors
    int *spart;               // SS_SCAN_BLOCKS partial sums of the scan of hist2, then their offsets
    double *pfirst, *plast;   // per piece of DS_PIECE sorted points: sums of its first and last run (d each)
};
constexpr int BF_CHUNK = 4096;        // points per step of the bound filter (256 threads x 16)
constexpr int SS_NB = 1024;           // one-wave blocks of the stable counting sorts
constexpr int SS_SCAN_BLOCKS = 1024;  // workgroups of the scan of their (key, block) table
constexpr int DS_PIECE = 512;         // sorted points per wave of the fixed-order centroid sums

// ---------------------------------------------------------------- rounding
// (selects rather than branches: these sit in the innermost loops)
__device__ __forceinline__ float f_up(float f)
{
    const unsigned u = __float_as_uint(f);
    const unsigned r = f > 0.f ? u + 1u : (f < 0.f ? u - 1u : 1u);
    return f < __builtin_huge_valf() ? __uint_as_float(r) : f;   // +inf, nan unchanged
}
__device__ __forceinline__ float f_dn(float f)
{
    const unsigned u = __float_as_uint(f);
    const unsigned r = f > 0.f ? u - 1u : (f < 0.f ? u + 1u : 0x80000001u);
    return f > -__builtin_huge_valf() ? __uint_as_float(r) : f;  // -inf, nan unchanged
}
// One step down / up for values whose exact counterpart is known to be >= 0
// (sums of non-negative terms, square roots): the result bounds the exact
// value from below / above.  Non-positive and NaN inputs give 0 / stay.
__device__ __forceinline__ float dn_nonneg(float x)
{
    return x > 0.f ? __uint_as_float(__float_as_uint(x) - 1u) : 0.f;
}
__device__ __forceinline__ float up_nonneg(float x)
{
    return x < __builtin_huge_valf() ? __uint_as_float(__float_as_uint(fmaxf(x, 0.f)) + 1u) : x;
}
// FP64 -> FP32 rounded toward +inf / -inf.
__device__ __forceinline__ float d2f_up(double v)
{
    float f = (float)v;
    return ((double)f < v) ? f_up(f) : f;
}
__device__ __forceinline__ float d2f_dn(double v)
{
    float f = (float)v;
    return ((double)f > v) ? f_dn(f) : f;
}

// BF16 round-to-nearest-even of a finite FP32 value.
__device__ __forceinline__ uint16_t f2bf(float f)
{
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((unsigned)h) << 16); }

// ------------------------------------------------------- offset-form bounds
// (each FP32 operation rounds to nearest; the f_up / f_dn step covers it)
__device__ __forceinline__ float ub_now(float u, float scu) { return f_up(u + scu); }
__device__ __forceinline__ float lb_now(float v, float sgu) { return f_dn(v - sgu); }
__device__ __forceinline__ float store_u(float ub, float scd) { return f_up(ub - scd); }
__device__ __forceinline__ float store_lb(float lb, float sgd) { return f_dn(lb + sgd); }
// Group q may hold the nearest centroid unless ub < lb_q now, i.e. unless
// ub + Sg[q] < v_q; s + one ulp bounds the exact sum from above (s >= 0).
__device__ __forceinline__ bool group_open(float ub, float sgu, float v)
{
    const float s = ub + sgu;
    return !(__uint_as_float(__float_as_uint(s) + 1u) < v);
}

// ------------------------------------------------- FP16 lower-bound codes
// BF16 mode can store each offset-form lower bound v as an FP16 code: the
// FP16 number at or below max(v, 0) * 2^-e, with 2^e a power-of-two scale
// chosen from the data at init so that distances land near 2^10.  Half the
// bytes of FP32 in the bound rows that the group filter and the recheck
// stream, at up to 2^-10 (relative) looser bounds.  The code truncates the
// FP32 significand (toward zero), flushes values below the FP16 normal
// range to 0 and saturates values above it at the largest finite FP16;
// decoding is exact.  A decoded code therefore never exceeds the bound it
// came from (raising a negative bound to 0 is valid: distances are >= 0).
__device__ __forceinline__ uint16_t lb16_enc(float v, float inv)
{
    const float w = fmaxf(v * inv, 0.f);   // NaN gives 0; the product is exact above FP32 subnormals
    const int c = (int)(__float_as_uint(w) >> 13) - (112 << 10);   // exponent rebias 127 -> 15
    return (uint16_t)min(max(c, 0), 0x7BFF);
}
__device__ __forceinline__ float lb16_dec(unsigned short b, float sc)
{
    return (float)__builtin_bit_cast(_Float16, b) * sc;
}

// ------------------------------------------------------- error bounds
// FP32 direct-form squared distance: four accumulators (coordinate i goes to
// accumulator i mod 4, fused multiply-add in coordinate order), combined as
// (a0 + a1) + (a2 + a3).  With m = ceil(d / 4) terms per accumulator the
// relative error of the result is below (m + 4) u, u = 2^-24 (rounded
// difference squared: 2u; m fused adds; two combining adds).  The bound used
// doubles the margin.  The same constant covers the 16-lane tree of the
// recheck (d/16 sequential terms and four combining levels).
__host__ __device__ __forceinline__ double eps2_direct(int d)
{
    return (double)((d + 3) / 4 + 8) * 5.9604644775390625e-08;   // * 2^-24
}
// Upper / lower bound on the true distance from a direct-form FP32 d^2 with
// relative error eps2, widened by rho (rho = 0 for FP32 inputs; the BF16
// rounding residuals of both vectors otherwise).
__device__ __forceinline__ float dist_hi(float d2, double eps2, double rho = 0.0)
{
    return d2f_up((sqrt((double)d2 * (1.0 + eps2)) + rho) * (1.0 + 0x1p-46));
}
__device__ __forceinline__ float dist_lo(float d2, double eps2, double rho = 0.0)
{
    if (!(d2 < __builtin_huge_valf())) return d2;
    const double v = (double)d2 * (1.0 - eps2);
    const double r = (v > 0.0 ? sqrt(v) * (1.0 - 0x1p-46) : 0.0) - rho;
    return r > 0.0 ? d2f_dn(r * (1.0 - 0x1p-46)) : 0.f;
}
// Error bound of the BF16x3 estimates (the distance calculator of Section 1
// must return what standard K-means returns, Abstract).  Products: rounding to
// nearest with 8-bit significands splits x = xh + xl + rx with
// |xl_i| <= 2^-8 (1 + 2^-8) |x_i| and |rx_i| <= 2^-16 |x_i|, and a centroid
// row c the same way.  With u = 2^-24, A >= ||x||, C >= ||c||:
//   |xh.ch + xl.ch + xh.cl - x.c| <= |xl.cl| + |rx.c| + |xh.rc| + |xl.rc|
//                                  <= 3.02 * 2^-16 A C
// hh = xh.ch sums ldb exact products in FP32 on the matrix cores; xl.ch and
// xh.cl (2 ldb products of size <= 2^-8 (1.01) |x_i c_i|) sum in two more
// accumulators, added once:
//   gamma_ldb (1.01) A C + gamma_2ldb 2^-7 (1.01) A C, doubled for the
//   unspecified summation order inside the matrix cores: <= 2.1 (ldb + 2) u A C
//   the adds forming S (two are allowed for): <= 2.05 u A C
// so |S - x.c| <= kappa A C, kappa = 3.02 2^-16 + 2.1 (ldb + 2) u + 2.05 u.
//
// Estimates relative to an anchor.  The chunk rows are not c_j but
// c~_j = fl(c_j - c_f), f the chunk's first slot (row f itself keeps c_f),
// and a tile of points may be taken relative to an anchor centroid r = c_a:
// x~ = fl(x - r), w~ = fl(c_f - r) staged as the chunk's first row, and
//   v = fl(fl(xn + Q_j) - 2 S),  S = fl(x~.c~_j + x~.w~)   (S = x~.w~ for j = f)
// with xn the squared norm of x~ (FP64 sum rounded) and Q_j = ||c_j - r||^2
// (FP64, rounded).  Without an anchor r = 0: x~ = x, w~ = c_f and Q_j =
// ||c_j||^2.  With A >= ||x~||, W >= ||w~|| and N_j >= ||c~_j||, B_j = W + N_j
// (the triangle inequality gives ||c_j - r|| <= B_j as well), the errors add
// up to
//   rounding of x~ and of w~ + c~_j: (2u + u^2) A^2 + 4.04 u A B_j
//   the two products and the added S: 2 (kappa + 1.01 u) A B_j
//   xn, Q_j, their sum and the final fused multiply-add: 1.01 u each, of
//     A^2, B_j^2, A^2 + B_j^2 and (A + B_j)^2
// and the bounds L = fl(v - e), U = fl(v + e) formed from v round once more
// (1.01 u (A + B_j)^2), so with
//   a = 6.05 u,  b = 2 kappa + 10.1 u,  c = 4.04 u
// and e_j = a A^2 + b A B_j + c B_j^2, both L <= ||x - c_j||^2 <= U hold.
// The kernels order rows by L with its low 4 significand bits cleared (the
// row's index rides there); clearing only lowers a non-negative L, so it
// stays a lower bound.
// Per row this is evaluated as e_j = E0 + N_j (h + c N_j) from the chunk's
// E0 = a A^2 + b A W + c W^2 and h = b A + 2 c W (every term is
// nonnegative; the coefficients' margin covers the rounding of these FP32
// operations).
// Relative to an anchor near the point (its assigned centroid), A is the
// distance to it and W, N_j distances between nearby centroids, so e_j shrinks
// with the cell sizes instead of the norms, row by row.
struct Eta3 {
    float a, b;
};
__host__ __device__ __forceinline__ double mfma_eta3_scale() { return (1.0 + 0x1p-20) * (1.0 + 0x1p-16); }
__device__ __forceinline__ Eta3 mfma_eta3_coef(int ldb)
{
    const double u = 5.9604644775390625e-08;
    const double kappa = 3.02 * 0x1p-16 + 2.1 * (double)(ldb + 2) * u + 2.05 * u;
    Eta3 k;
    k.a = d2f_up(6.05 * u * mfma_eta3_scale());
    k.b = d2f_up((2.0 * kappa + 10.1 * u) * mfma_eta3_scale());
    return k;
}
__host__ __device__ __forceinline__ double mfma_eta3_c() { return 4.04 * 5.9604644775390625e-08 * mfma_eta3_scale(); }
// A >= ||x~|| from its squared norm rounded to FP32, once per point.
__device__ __forceinline__ float mfma_eta3_a(float xn) { return d2f_up(sqrt((double)xn) * (1.0 + 0x1p-22)); }
// c and 2 c as FP32 constants, rounded up (2 c exactly twice c).
constexpr float ETA3_C = (float)(4.04 * 0x1p-24 * (1.0 + 0x1p-20) * (1.0 + 0x1p-16) * (1.0 + 0x1p-22));
constexpr float ETA3_C2 = 2.f * ETA3_C;
// Per point: (b A, a A^2).
__device__ __forceinline__ float2 mfma_eta3_pt(const Eta3 &k, float A) { return make_float2(k.b * A, k.a * (A * A)); }
// A chunk's (W, c W^2), the second rounded up (the tables hold it).
__device__ __forceinline__ float2 mfma_eta3_w(float W)
{
    return make_float2(W, d2f_up(mfma_eta3_c() * (double)W * (double)W * (1.0 + 0x1p-50)));
}

// --------------------------------------------------- tuple merge (d^2, slot, second)
struct Best3 {
    float m1;
    int s1;
    float m2;
};
__device__ __forceinline__ Best3 merge3(Best3 a, Best3 b)
{
    // b wins on a smaller value, or an equal value at a lower slot (within one
    // group slots are in ascending original index, so this is the tie rule).
    const bool nb = (b.m1 < a.m1) || (b.m1 == a.m1 && b.s1 < a.s1);
    Best3 r;
    r.m2 = nb ? fminf(a.m1, b.m2) : fminf(a.m2, b.m1);
    r.m1 = nb ? b.m1 : a.m1;
    r.s1 = nb ? b.s1 : a.s1;
    return r;
}
__device__ __forceinline__ Best3 shfl_xor3(Best3 v, int mask)
{
    Best3 r;
    r.m1 = __shfl_xor(v.m1, mask);
    r.s1 = __shfl_xor(v.s1, mask);
    r.m2 = __shfl_xor(v.m2, mask);
    return r;
}

// ------------------------------------------------------------- wave helpers
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (WAVE - 1)); }

// Append the lanes with `pred` to a list guarded by a 64-bit counter; every
// lane of the wave must call it.  Returns the slot of the calling lane, or -1.
__device__ __forceinline__ long long wave_append(unsigned long long *ctr, bool pred)
{
    const unsigned long long m = __ballot(pred);
    if (m == 0ull) return -1;
    const int lane = lane_id();
    const int leader = __ffsll((long long)m) - 1;
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(ctr, (unsigned long long)__popcll(m));
    const unsigned lo = __shfl((unsigned)(base & 0xFFFFFFFFull), leader);
    const unsigned hi = __shfl((unsigned)(base >> 32), leader);
    base = ((unsigned long long)hi << 32) | lo;
    if (!pred) return -1;
    return (long long)(base + __popcll(m & ((1ull << lane) - 1ull)));
}

__device__ __forceinline__ float wave_min(float v)
{
    for (int o = 32; o >= 1; o >>= 1) v = fminf(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_sum_d(double v)
{
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

}  // namespace kp
