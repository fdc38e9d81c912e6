/* The FP64 oracle (test infrastructure) under AddressSanitizer and
 * UndefinedBehaviorSanitizer: every entry point on small random inputs,
 * single- and multi-threaded, with checks that need no second
 * implementation (labels in range, each point's distance to its label is
 * the smallest, the update is the mean, SSE never rises over Lloyd
 * iterations, empty clusters keep their centroid). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void kpo_assign(const float *X, int64_t n, int d, const double *C, int k, int32_t *labels, double *dmin2,
                double *dsec2, int nthreads);
void kpo_dist2_to(const float *X, int64_t n, int d, const double *C, const int32_t *labels, double *out,
                  int nthreads);
void kpo_update(const float *X, int64_t n, int d, const int32_t *labels, int k, const double *Cprev, double *Cnew,
                int64_t *counts, int nthreads);
double kpo_sse(const float *X, int64_t n, int d, const double *C, const int32_t *labels, int nthreads);
void kpo_lloyd(const float *X, int64_t n, int d, const double *C0, int k, int T, int32_t *labels_out, double *C_out,
               double *sse_assign, double *sse_update, double *C_final, int nthreads);

static int fails = 0;
#define CHECK(c)                                                            \
    do {                                                                    \
        if (!(c)) {                                                         \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++fails;                                                        \
        }                                                                   \
    } while (0)

static uint64_t st = 88172645463325252ull;
static double unif(void)
{
    st ^= st << 13;
    st ^= st >> 7;
    st ^= st << 17;
    return (double)(st >> 11) * 0x1.0p-53;
}

static void run(int64_t n, int d, int k, int T, int nthreads)
{
    float *X = malloc(sizeof(float) * (size_t)n * d);
    double *C0 = malloc(sizeof(double) * (size_t)k * d), *C1 = malloc(sizeof(double) * (size_t)k * d);
    double *Cf = malloc(sizeof(double) * (size_t)k * d), *Cs = malloc(sizeof(double) * (size_t)T * k * d);
    int32_t *lab = malloc(sizeof(int32_t) * (size_t)n), *labs = malloc(sizeof(int32_t) * (size_t)T * n);
    double *dmin = malloc(sizeof(double) * (size_t)n), *dsec = malloc(sizeof(double) * (size_t)n);
    double *dto = malloc(sizeof(double) * (size_t)n);
    double *sa = malloc(sizeof(double) * (size_t)T), *su = malloc(sizeof(double) * (size_t)T);
    int64_t *cnt = malloc(sizeof(int64_t) * (size_t)k);
    for (int64_t i = 0; i < n * d; ++i) X[i] = (float)(unif() * 20.0 - 10.0);
    for (int64_t i = 0; i < (int64_t)k * d; ++i) C0[i] = unif() * 20.0 - 10.0;
    if (k > 1)   /* a centroid far from every point: its cluster stays empty */
        for (int i = 0; i < d; ++i) C0[(int64_t)(k - 1) * d + i] = 1e6;

    kpo_assign(X, n, d, C0, k, lab, dmin, dsec, nthreads);
    kpo_dist2_to(X, n, d, C0, lab, dto, nthreads);
    for (int64_t p = 0; p < n; ++p) {
        CHECK(lab[p] >= 0 && lab[p] < k);
        CHECK(dto[p] == dmin[p] && dmin[p] <= dsec[p]);
    }
    kpo_update(X, n, d, lab, k, C0, C1, cnt, nthreads);
    int64_t tot = 0;
    for (int j = 0; j < k; ++j) {
        tot += cnt[j];
        if (cnt[j] == 0)
            for (int i = 0; i < d; ++i) CHECK(C1[(int64_t)j * d + i] == C0[(int64_t)j * d + i]);
    }
    CHECK(tot == n);
    if (k > 1) CHECK(cnt[k - 1] == 0);
    /* the mean of cluster lab[0], summed here in point order */
    for (int i = 0; i < d; ++i) {
        double s = 0.0;
        for (int64_t p = 0; p < n; ++p)
            if (lab[p] == lab[0]) s += X[p * d + i];
        const double m = s / (double)cnt[lab[0]];
        CHECK(fabs(m - C1[(int64_t)lab[0] * d + i]) <= 1e-12 * (1.0 + fabs(m)));
    }
    const double e0 = kpo_sse(X, n, d, C0, lab, nthreads), e1 = kpo_sse(X, n, d, C1, lab, nthreads);
    CHECK(e1 <= e0 * (1.0 + 1e-12));

    kpo_lloyd(X, n, d, C0, k, T, labs, Cs, sa, su, Cf, nthreads);
    for (int t = 0; t < T; ++t) {
        CHECK(su[t] <= sa[t] * (1.0 + 1e-12));
        if (t > 0) CHECK(sa[t] <= su[t - 1] * (1.0 + 1e-12));
    }
    for (int64_t i = 0; i < (int64_t)k * d; ++i) CHECK(Cf[i] == Cs[(int64_t)(T - 1) * k * d + i]);
    free(X); free(C0); free(C1); free(Cf); free(Cs); free(lab); free(labs);
    free(dmin); free(dsec); free(dto); free(sa); free(su); free(cnt);
}

int main(void)
{
    const int threads[2] = {1, 4};
    for (int t = 0; t < 2; ++t) {
        run(1, 1, 1, 2, threads[t]);
        run(7, 3, 2, 3, threads[t]);
        run(1000, 8, 16, 5, threads[t]);
        run(777, 33, 40, 4, threads[t]);
    }
    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("oracle checks passed\n");
    return 0;
}
