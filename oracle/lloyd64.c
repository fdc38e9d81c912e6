/*
 * CPU FP64 oracle for the filtered K-means path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  The GPU library shares no code with it.
 *
 * What it computes: standard K-means (Lloyd's algorithm), the computation
 * the paper accelerates and the one its filters must reproduce exactly
 * (Abstract; Section 1, which names the multi-level filters as a way of
 * skipping distance computations without changing the result; Section 2
 * compares against "standard K-means").  The paper prints no formula, so
 * each step below is the textbook definition:
 *
 *   assign:  a(x) = argmin_j  sum_i (x_i - c_{j,i})^2, lowest j on ties
 *   update:  c_j  = (sum_{a(x)=j} x) / n_j, unchanged when n_j = 0
 *
 * Everything is FP64 in direct (difference-of-coordinates) form.  The FP32
 * inputs are promoted exactly.  OpenMP parallelises over points only; each
 * point's sum runs in coordinate order, so results do not depend on the
 * thread count, except the SSE and update sums, which are reduced per
 * thread and then added in thread order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    return omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

int kpo_threads(int nthreads) { return set_threads(nthreads); }

/* Squared Euclidean distance in FP64, direct form, coordinates in order. */
static double dist2(const float *x, const double *c, int d)
{
    double s = 0.0;
    for (int i = 0; i < d; ++i) {
        double t = (double)x[i] - c[i];
        s += t * t;
    }
    return s;
}

/* Assignment step: nearest centroid per point (lowest index on exact ties).
 * X: n*d FP32 row-major; C: k*d FP64 row-major.
 * labels[n] (int32) and dmin2[n] (FP64 squared distance) are written;
 * dsec2[n], when not NULL, receives the second-smallest squared distance
 * (+inf when k == 1). */
void kpo_assign(const float *X, int64_t n, int d, const double *C, int k,
                int32_t *labels, double *dmin2, double *dsec2, int nthreads)
{
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        const float *x = X + p * (int64_t)d;
        double best = INFINITY, second = INFINITY;
        int32_t arg = -1;
        for (int j = 0; j < k; ++j) {
            double v = dist2(x, C + (int64_t)j * d, d);
            if (v < best) {          /* strict: an equal later j never wins */
                second = best;
                best = v;
                arg = j;
            } else if (v < second) {
                second = v;
            }
        }
        labels[p] = arg;
        if (dmin2) dmin2[p] = best;
        if (dsec2) dsec2[p] = second;
    }
}

/* Squared distance of every point to the centroid its label names. */
void kpo_dist2_to(const float *X, int64_t n, int d, const double *C,
                  const int32_t *labels, double *out, int nthreads)
{
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p)
        out[p] = dist2(X + p * (int64_t)d, C + (int64_t)labels[p] * d, d);
}

/* Update step: FP64 means of the points assigned to each centroid.
 * Cprev supplies the value of a centroid that received no point.
 * counts[k] (int64) receives n_j. */
void kpo_update(const float *X, int64_t n, int d, const int32_t *labels, int k,
                const double *Cprev, double *Cnew, int64_t *counts, int nthreads)
{
    int nt = set_threads(nthreads);
    double *part = (double *)calloc((size_t)nt * k * d, sizeof(double));
    int64_t *pcnt = (int64_t *)calloc((size_t)nt * k, sizeof(int64_t));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *S = part + (size_t)tid * k * d;
        int64_t *cn = pcnt + (size_t)tid * k;
#pragma omp for schedule(static)
        for (int64_t p = 0; p < n; ++p) {
            int j = labels[p];
            const float *x = X + p * (int64_t)d;
            double *s = S + (int64_t)j * d;
            for (int i = 0; i < d; ++i) s[i] += (double)x[i];
            cn[j] += 1;
        }
    }
    for (int j = 0; j < k; ++j) {
        int64_t cnt = 0;
        for (int t = 0; t < nt; ++t) cnt += pcnt[(size_t)t * k + j];
        counts[j] = cnt;
        for (int i = 0; i < d; ++i) {
            if (cnt == 0) {
                Cnew[(int64_t)j * d + i] = Cprev[(int64_t)j * d + i];
            } else {
                double s = 0.0;
                for (int t = 0; t < nt; ++t) s += part[((size_t)t * k + j) * d + i];
                Cnew[(int64_t)j * d + i] = s / (double)cnt;
            }
        }
    }
    free(part);
    free(pcnt);
}

/* Sum of squared distances of every point to its labelled centroid. */
double kpo_sse(const float *X, int64_t n, int d, const double *C,
               const int32_t *labels, int nthreads)
{
    set_threads(nthreads);
    double total = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : total)
    for (int64_t p = 0; p < n; ++p)
        total += dist2(X + p * (int64_t)d, C + (int64_t)labels[p] * d, d);
    return total;
}

/* T iterations of Lloyd from C0.  One iteration = one assignment step with
 * the current centroids, then one update step.  For t = 0..T-1:
 *   labels_out[t*n ..]  (may be NULL)   the assignment of iteration t+1
 *   C_out[t*k*d ..]     (may be NULL)   the centroids after iteration t+1
 *   sse_assign[t]       (may be NULL)   SSE of that assignment, old centroids
 *   sse_update[t]       (may be NULL)   SSE of that assignment, new centroids
 * C_final[k*d] receives the final centroids. */
void kpo_lloyd(const float *X, int64_t n, int d, const double *C0, int k, int T,
               int32_t *labels_out, double *C_out, double *sse_assign,
               double *sse_update, double *C_final, int nthreads)
{
    double *C = (double *)malloc(sizeof(double) * (size_t)k * d);
    double *Cn = (double *)malloc(sizeof(double) * (size_t)k * d);
    int32_t *lab = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
    memcpy(C, C0, sizeof(double) * (size_t)k * d);
    for (int t = 0; t < T; ++t) {
        kpo_assign(X, n, d, C, k, lab, NULL, NULL, nthreads);
        if (sse_assign) sse_assign[t] = kpo_sse(X, n, d, C, lab, nthreads);
        kpo_update(X, n, d, lab, k, C, Cn, cnt, nthreads);
        if (sse_update) sse_update[t] = kpo_sse(X, n, d, Cn, lab, nthreads);
        if (labels_out) memcpy(labels_out + (int64_t)t * n, lab, sizeof(int32_t) * (size_t)n);
        if (C_out) memcpy(C_out + (int64_t)t * k * d, Cn, sizeof(double) * (size_t)k * d);
        double *tmp = C; C = Cn; Cn = tmp;
    }
    memcpy(C_final, C, sizeof(double) * (size_t)k * d);
    free(C);
    free(Cn);
    free(lab);
    free(cnt);
}
