// Device-side data layout and numeric helpers of the filtered K-means library.
//
// Layout in HBM (per problem, all carved from the caller's workspace):
//   X      n x d   FP32  caller's points, row-major, borrowed
//   Xb     n x ldb BF16  round-to-nearest-even shadow of X, zero-padded to
//                        ldb = roundup(d, 32) (BF16 mode only)
//   xn     n       FP32  ||Xb_i||^2 (BF16 mode)
//   xr     n       FP32  ||X_i - Xb_i|| rounded up (BF16 mode)
//   st     n       16 B  PointState: assignment slot, upper bound, point-level
//                        lower bound, stamp of the last refresh
//   lb     n x gs  FP32  group-level lower bounds, gs = roundup(g, 4)
//   centroids in "slot" order: the members of group q occupy slots
//   gstart[q] .. gstart[q] + gsize[q] - 1 in ascending original index, and the
//   group is padded with empty slots to a multiple of 16 so that every
//   16-slot chunk of a MFMA tile belongs to one group.
//
// Bounds are stored "lazily": the drift of the centroids is accumulated in
// FP64 ring buffers (per slot, per group and its maximum) and a point's
// stored bounds are brought to the current iteration only when the point is
// looked at.  Exact arithmetic gives the same bounds as updating every point
// in every iteration; the rounding directions below keep them valid.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kp {

constexpr int WAVE = 64;
constexpr int CHUNK = 16;             // centroid slots per MFMA tile / group padding
constexpr int STATS_CAP = 1024;       // per-iteration stats ring
constexpr int NCTR = 8;               // per-iteration counters

// counters (unsigned long long) per problem
enum { CTR_L1 = 0, CTR_L3 = 1, CTR_MOVED = 2, CTR_PAIRS = 3, CTR_DIST = 4, CTR_DENSE = 5 };

struct __attribute__((aligned(16))) PointState {
    int a;        // slot of the assigned centroid
    float ub;     // upper bound on d(x, c_a), valid at stamp tx (see ub_eff)
    float lbp;    // lower bound on min_{j != a} d(x, c_j) at stamp tx
    int tx;       // iteration whose assignment step last refreshed the bounds
};

typedef __bf16 bf16x8 __attribute__((__vector_size__(8 * sizeof(__bf16))));
typedef float f32x4 __attribute__((__vector_size__(4 * sizeof(float))));

struct ProbDev {
    int64_t n;
    int d, k, g, kg;          // kg = number of slots (with padding)
    int ldc, ldb, gs;         // leading dims: c32 (roundup 4), bf16 (roundup 32), lb row
    int prec;                 // 0 fp32 direct, 1 bf16 + recheck
    int W;                    // ring length (age limit)
    int maxgs;                // largest group size (real members)
    int pad0;
    const float *X;
    uint16_t *Xb;
    float *xn, *xr;
    PointState *st;
    float *lb;
    float *c32;
    uint16_t *cb;
    float *cn, *cr;
    double *c64, *sums, *delta;
    int *cnt;
    const int *perm;          // slot -> original index, -1 for padding
    const int *slot_group;    // slot -> group, -1 for padding
    const int *gstart, *gsize;
    double *Sc, *Sg, *Sd;     // rings: W x kg, W x g, W
    int *L1;                  // point ids failing the point-level filter
    int4 *L3;                 // (point, old slot, bits of U*, flags) for the FP32 recheck
    int *mv_pt, *mv_old, *mv_new;   // moved points
    int *srt_pt, *srt_key;    // entries sorted by centroid slot (sign in bit 31 of srt_pt)
    int *hist, *cursor;       // kg + 1
    unsigned long long *ctr;  // NCTR counters of the running iteration
    long long *stats;         // STATS_CAP x 8
    int *iter;                // completed iterations
    float *scal;              // [0] max ||c_hat||, [1] max ||c - c_hat||
};

// ---------------------------------------------------------------- rounding
__device__ __forceinline__ float f_up(float f)
{
    if (!(f < __builtin_huge_valf())) return f;                  // +inf, nan
    unsigned u = __float_as_uint(f);
    if (f > 0.f) u += 1u; else if (f < 0.f) u -= 1u; else u = 1u;
    return __uint_as_float(u);
}
__device__ __forceinline__ float f_dn(float f)
{
    if (!(f > -__builtin_huge_valf())) return f;
    unsigned u = __float_as_uint(f);
    if (f > 0.f) u -= 1u; else if (f < 0.f) u += 1u; else u = 0x80000001u;
    return __uint_as_float(u);
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

// ------------------------------------------------------- error bounds
// FP32 direct-form squared distance: four accumulators (coordinate i goes to
// accumulator i mod 4, fused multiply-add in coordinate order), combined as
// (a0 + a1) + (a2 + a3).  With m = ceil(d / 4) terms per accumulator the
// relative error of the result is below (m + 4) u, u = 2^-24 (rounded
// difference squared: 2u; m fused adds; two combining adds).  EPS2 doubles
// the margin.
__host__ __device__ __forceinline__ double eps2_direct(int d)
{
    return (double)((d + 3) / 4 + 8) * 5.9604644775390625e-08;   // * 2^-24
}
// Upper / lower bound on the true distance from a direct-form FP32 d^2.
__device__ __forceinline__ float dist_hi(float d2, double eps2)
{
    return d2f_up(sqrt((double)d2 * (1.0 + eps2)) * (1.0 + 0x1p-46));
}
__device__ __forceinline__ float dist_lo(float d2, double eps2)
{
    double v = (double)d2 * (1.0 - eps2);
    return v > 0.0 ? d2f_dn(sqrt(v) * (1.0 - 0x1p-46)) : 0.f;
}
// BF16 MFMA estimate v = ||xb||^2 + ||cb||^2 - 2 xb.cb of ||xb - cb||^2:
//   | v - ||xb - cb||^2 | <= eta,  | ||xb - cb|| - ||x - c|| | <= rho,
// so the true distance lies in [sqrt(max(v - eta, 0)) - rho, sqrt(v + eta) + rho].
__device__ __forceinline__ float mfma_hi(float v, double eta, double rho)
{
    double t = (double)v + eta;
    return d2f_up((sqrt(t > 0.0 ? t : 0.0) + rho) * (1.0 + 0x1p-46));
}
__device__ __forceinline__ float mfma_lo(float v, double eta, double rho)
{
    if (!(v < __builtin_huge_valf())) return v;
    double t = (double)v - eta;
    double s = t > 0.0 ? sqrt(t) * (1.0 - 0x1p-46) : 0.0;
    double r = s - rho;
    return r > 0.0 ? d2f_dn(r * (1.0 - 0x1p-46)) : 0.f;
}
// eta of one point: the products of BF16 values are exact in FP32, so the
// MFMA dot product carries at most gamma_ldb * ||xb|| ||cb||; the FP32 norms
// carry u ||.||^2 each and the two final operations 2u (||xb|| + ||cb||)^2.
// Everything is below (ldb + 4) u (||xb|| + ||cb||)^2; a factor 2 covers the
// undocumented internal accumulation order of the matrix cores.
__device__ __forceinline__ double mfma_eta(float xn, float bmax, int ldb)
{
    double a = sqrt((double)xn) + (double)bmax;
    return 2.0 * (double)(ldb + 4) * 5.9604644775390625e-08 * a * a * (1.0 + 0x1p-20);
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
    bool nb = (b.m1 < a.m1) || (b.m1 == a.m1 && b.s1 < a.s1);
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
    unsigned long long m = __ballot(pred);
    if (m == 0ull) return -1;
    int lane = lane_id();
    int leader = __ffsll((long long)m) - 1;
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(ctr, (unsigned long long)__popcll(m));
    unsigned lo = __shfl((unsigned)(base & 0xFFFFFFFFull), leader);
    unsigned hi = __shfl((unsigned)(base >> 32), leader);
    base = ((unsigned long long)hi << 32) | lo;
    if (!pred) return -1;
    return (long long)(base + __popcll(m & ((1ull << lane) - 1ull)));
}

__device__ __forceinline__ float wave_min(float v)
{
    for (int o = 32; o >= 1; o >>= 1) v = fminf(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ float wave_max(float v)
{
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_sum_d(double v)
{
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Lazily accumulated drift between stamp tx and iteration t: the bounds stored
// at tx were valid for the centroids used by iteration tx; the ring holds the
// cumulative drift S(tau) after update tau at index tau mod W.  The result
// is rounded up (every FP64 rounding error is below 2^-52 of the larger sum).
__device__ __forceinline__ double drift_between(const double *ring, int stride, int idx, int t, int tx, int W)
{
    double now = ring[(size_t)((t - 1) % W) * stride + idx];
    double then = ring[(size_t)((tx - 1) % W) * stride + idx];
    return (now - then) + now * 0x1p-44;
}
// The same difference rounded down (never below zero).
__device__ __forceinline__ double drift_between_dn(const double *ring, int stride, int idx, int t, int tx, int W)
{
    double now = ring[(size_t)((t - 1) % W) * stride + idx];
    double then = ring[(size_t)((tx - 1) % W) * stride + idx];
    double v = (now - then) - now * 0x1p-44;
    return v > 0.0 ? v : 0.0;
}
// An upper bound stored at tx, moved to iteration t (FP64, rounded up).
__device__ __forceinline__ double up_eff(float stored, double drift)
{
    double v = (double)stored + drift;
    return v + fabs(v) * 0x1p-50;
}
// A lower bound stored at tx, moved to iteration t (FP64, rounded down).
__device__ __forceinline__ double lo_eff(float stored, double drift)
{
    double v = (double)stored - drift;
    return v - fabs(v) * 0x1p-50;
}

}  // namespace kp
