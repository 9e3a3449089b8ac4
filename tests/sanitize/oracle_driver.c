/*
 * Sanitizer driver of the FP64 oracle (test infrastructure): built with
 * AddressSanitizer and UndefinedBehaviorSanitizer together with
 * oracle/haar_oracle.c and run by tests/test_sanitizers.py.  It calls every
 * oracle entry point on small odd and even sizes, every depth and a batch of
 * items, so that an out-of-bounds access, a use of uninitialised scratch
 * that ASan can see, or undefined integer/shift behaviour ends the run with
 * a report.  It also checks the two identities that need no reference
 * values: the synthesis inverts the analysis, and the direct bank equals the
 * fast bank.  Exit status 0 means every call was clean.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void oracle_fwd_1d(const double* x, double* y, int64_t n, int32_t levels, int64_t batch);
void oracle_inv_1d(const double* y, double* x, int64_t n, int32_t levels, int64_t batch);
void oracle_direct_fwd_1d(const double* x, double* y, int64_t n, int32_t levels, int64_t batch);
void oracle_direct_inv_1d(const double* y, double* x, int64_t n, int32_t levels, int64_t batch);
void oracle_fwd_2d(const double* x, double* y, int64_t h, int64_t w, int32_t levels, int64_t batch);
void oracle_inv_2d(const double* y, double* x, int64_t h, int64_t w, int32_t levels, int64_t batch);
void oracle_fwd_3d(const double* x, double* y, int64_t d, int64_t h, int64_t w, int32_t levels,
                   int64_t batch);
void oracle_inv_3d(const double* y, double* x, int64_t d, int64_t h, int64_t w, int32_t levels,
                   int64_t batch);
void oracle_shrink_1d(const double* x, double* y, int64_t n, int32_t levels, int64_t batch,
                      int32_t mode, const double* thr);
void oracle_shrink_2d(const double* x, double* y, int64_t h, int64_t w, int32_t levels,
                      int64_t batch, int32_t mode, const double* thr);
void oracle_l1_grad_2d(const double* x, double* g, double* loss, int64_t h, int64_t w,
                       int32_t levels, int64_t batch);
void oracle_filter_taps(double b0[2], double b1[2], double a0[2], double a1[2]);

static uint64_t state = 0x9e3779b97f4a7c15ull;
static double rnd(void) {           /* xorshift64*, uniform in [-1, 1) */
    state ^= state >> 12;
    state ^= state << 25;
    state ^= state >> 27;
    return (double)((state * 0x2545f4914f6cdd1dull) >> 11) / 4503599627370496.0 - 1.0;
}

static int levels_of(int64_t n) {
    int L = 0;
    while (((int64_t)1 << L) < n) ++L;
    return L;
}

static double* make(int64_t n) {
    double* p = (double*)malloc((size_t)n * sizeof(double));
    for (int64_t i = 0; i < n; ++i) p[i] = rnd();
    return p;
}

static double maxdiff(const double* a, const double* b, int64_t n) {
    double m = 0.0;
    for (int64_t i = 0; i < n; ++i) m = fmax(m, fabs(a[i] - b[i]));
    return m;
}

static int failures = 0;
static void expect(int ok, const char* what, long long a, long long b, long long c) {
    if (!ok) {
        fprintf(stderr, "FAIL %s (%lld, %lld, %lld)\n", what, a, b, c);
        ++failures;
    }
}

int main(void) {
    const int64_t lens[] = {1, 2, 3, 5, 8, 31, 64, 100, 257};
    const int64_t batch = 3;
    for (size_t i = 0; i < sizeof lens / sizeof *lens; ++i) {
        const int64_t n = lens[i], tot = n * batch;
        for (int L = 0; L <= levels_of(n); ++L) {
            double *x = make(tot), *y = make(tot), *z = make(tot), *d = make(tot);
            oracle_fwd_1d(x, y, n, L, batch);
            oracle_inv_1d(y, z, n, L, batch);
            expect(maxdiff(x, z, tot) < 1e-12, "1d round trip", n, L, 0);
            oracle_direct_fwd_1d(x, d, n, L, batch);
            expect(maxdiff(y, d, tot) < 1e-12, "1d direct == fast", n, L, 0);
            oracle_direct_inv_1d(y, d, n, L, batch);
            expect(maxdiff(z, d, tot) < 1e-12, "1d direct inverse", n, L, 0);
            double thr[64];
            for (int j = 0; j < 64; ++j) thr[j] = 0.1 * (j + 1);
            oracle_shrink_1d(x, d, n, L, batch, 0, thr);
            oracle_shrink_1d(x, d, n, L, batch, 1, thr);
            free(x); free(y); free(z); free(d);
        }
    }
    const int64_t dims[][2] = {{1, 1}, {1, 7}, {7, 1}, {3, 5}, {8, 8}, {17, 33}, {40, 24}};
    for (size_t i = 0; i < sizeof dims / sizeof *dims; ++i) {
        const int64_t h = dims[i][0], w = dims[i][1], tot = h * w * batch;
        const int Lmax = levels_of(h > w ? h : w);
        for (int L = 0; L <= Lmax; ++L) {
            double *x = make(tot), *y = make(tot), *z = make(tot), *g = make(tot);
            double loss[3];
            oracle_fwd_2d(x, y, h, w, L, batch);
            oracle_inv_2d(y, z, h, w, L, batch);
            expect(maxdiff(x, z, tot) < 1e-12, "2d round trip", h, w, L);
            double thr[64];
            for (int j = 0; j < 64; ++j) thr[j] = 0.05 * (j + 1);
            oracle_shrink_2d(x, g, h, w, L, batch, 0, thr);
            oracle_shrink_2d(x, g, h, w, L, batch, 1, thr);
            if (L >= 1) oracle_l1_grad_2d(x, g, loss, h, w, L, batch);
            free(x); free(y); free(z); free(g);
        }
    }
    const int64_t vols[][3] = {{1, 1, 1}, {2, 3, 5}, {9, 4, 7}, {8, 8, 8}, {5, 17, 3}};
    for (size_t i = 0; i < sizeof vols / sizeof *vols; ++i) {
        const int64_t d = vols[i][0], h = vols[i][1], w = vols[i][2], tot = d * h * w * batch;
        int64_t m = d > h ? d : h;
        m = m > w ? m : w;
        for (int L = 0; L <= levels_of(m); ++L) {
            double *x = make(tot), *y = make(tot), *z = make(tot);
            oracle_fwd_3d(x, y, d, h, w, L, batch);
            oracle_inv_3d(y, z, d, h, w, L, batch);
            expect(maxdiff(x, z, tot) < 1e-12, "3d round trip", d * 10000 + h * 100 + w, L, 0);
            free(x); free(y); free(z);
        }
    }
    double b0[2], b1[2], a0[2], a1[2];
    oracle_filter_taps(b0, b1, a0, a1);
    if (failures) return 1;
    printf("oracle sanitizer driver: all calls clean\n");
    return 0;
}
