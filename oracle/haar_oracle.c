/*
 * FP64 oracle for the fast Haar wavelet transform (Ashok et al., "The Fast
 * Haar Wavelet Transform for Signal & Image Processing").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * CPU definition that the GPU library is checked against.  It is called only
 * by the test suite, by the smoke check and by the CPU-baseline leg of the
 * benchmark; the library's product path never links, loads or calls it, and
 * it shares no code, header or constant with the HIP sources.
 *
 * Everything is double precision.  No blocking, fusion or reordering beyond
 * what the definitions state.  Buffers are row-major and batch-major:
 *   1D: [batch][n]          2D: [batch][h][w]
 * Outputs are out-of-place and have the same size as the inputs.
 *
 * Definitions followed (section / equation of the paper):
 *   - Haar filters b0 = [1/sqrt2, 1/sqrt2], b1 from Eq. (9) (B00 - z^-1 B01),
 *     synthesis a0, a1 from Eq. (17)-(18), polyphase constant
 *     b00 = b01 = a00 = a01 = 1/sqrt2 (Sec. III after Eq. (12), Sec. IV
 *     after Eq. (19)).
 *   - Fast analysis bank (Sec. III, Eq. (11)-(12), Fig. 4): split the input
 *     into its two polyphase components first, then one sum and one
 *     difference per pair, scaled by b00:
 *         a[m] = b00 * (x[2m] + x[2m+1]),   d[m] = b00 * (x[2m+1] - x[2m]).
 *   - Fast synthesis bank (Sec. IV, Eq. (19), Fig. 7): even phase
 *     a00*(a - d), odd phase a01*(a + d), up-sampler moved to the output.
 *   - Direct ("original") bank of Fig. 1/Fig. 2: full-rate convolution with
 *     the two analysis filters followed by decimation, and up-sampling
 *     followed by convolution with the synthesis filters (Eq. (13)); kept
 *     here as an independent formulation that the fast bank must equal.
 *
 * Readings where the paper is silent (each is listed with its reason in the
 * design notes of the repository):
 *   - multi-level = dyadic recursion on the approximation only (Sec. I
 *     "hierarchically decomposing", Sec. V approximation/detail data);
 *   - packed layout [a_L | d_L | d_{L-1} | ... | d_1];
 *   - 2D = one 1D level along every row (width) of the current LL region,
 *     then along every column (height); bands LL (top-left), HL (top-right,
 *     high along width), LH (bottom-left, high along height), HH;
 *   - odd lengths ("carry rule"): when a level sees an odd count, its last
 *     sample passes unscaled into the approximation; there is no detail
 *     for it.  ceil(n/2) approximations, floor(n/2) details.
 *   - the sparsity loss of a training step through the 2D transform, sum of
 *     |details| + 0.5 ||LL_L||^2, and its gradient (the synthesis bank
 *     applied to the coefficient gradient, since W^T = W^-1);
 *   - 3D (volumes [batch][d][h][w], the paper's medical-image use): the 2D
 *     reading extended by one axis; per level one 1D level along x (width),
 *     then y (height), then z (depth) on the current LLL region, recursion
 *     on LLL; eight octant bands named by their (x, y, z) filters.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* b00 = a00 = 1/sqrt(2) in double precision (Sec. III, Sec. IV). */
static double b00(void) { return sqrt(0.5); }

/* ---------------------------------------------------------------------- */
/* One level of the fast analysis bank (Fig. 4) on n samples of a strided  */
/* line.  Output packed [a (ceil(n/2)) | d (floor(n/2))] on `out`.         */
/* `in` and `out` must not overlap.                                        */
/* ---------------------------------------------------------------------- */
static void fast_analysis_level(const double* in, int64_t si, double* out,
                                int64_t so, int64_t n)
{
    const double s = b00();
    const int64_t pairs = n / 2;          /* floor(n/2) details          */
    const int64_t na = n - pairs;         /* ceil(n/2) approximations    */
    for (int64_t m = 0; m < pairs; ++m) {
        const double x0 = in[(2 * m) * si];      /* even polyphase part  */
        const double x1 = in[(2 * m + 1) * si];  /* odd polyphase part   */
        out[m * so] = s * (x0 + x1);             /* Eq. (11)            */
        out[(na + m) * so] = s * (x1 - x0);      /* Eq. (12)            */
    }
    if (n & 1) out[pairs * so] = in[(n - 1) * si]; /* carry, unscaled    */
}

/* One level of the fast synthesis bank (Fig. 7): inverse of the above.  */
static void fast_synthesis_level(const double* in, int64_t si, double* out,
                                 int64_t so, int64_t n)
{
    const double s = b00();
    const int64_t pairs = n / 2;
    const int64_t na = n - pairs;
    for (int64_t m = 0; m < pairs; ++m) {
        const double a = in[m * si];
        const double d = in[(na + m) * si];
        out[(2 * m) * so] = s * (a - d);         /* even phase, Eq. (19) */
        out[(2 * m + 1) * so] = s * (a + d);     /* odd phase, Eq. (19)  */
    }
    if (n & 1) out[(n - 1) * so] = in[pairs * si]; /* carry, unscaled    */
}

/* ---------------------------------------------------------------------- */
/* The filter taps of the direct structure (Fig. 1/2, Fig. 5).           */
/* Causal FIR taps h[0] + h[1] z^-1.                                      */
/*   B0(z) = B00(z^2) + z^-1 B01(z^2)   Eq. (8)                          */
/*   B1(z) = B00(z^2) - z^-1 B01(z^2)   Eq. (9)                          */
/*   A0(z) = A00(z^2) + z^-1 A01(z^2)   Eq. (17)                         */
/*   A1(z) = -A00(z^2) + z^-1 A01(z^2)  Eq. (18)                         */
/* with all polyphase constants 1/sqrt2 and no factor 2 on the synthesis   */
/* side (unit-gain reading of Eq. (14)-(15)).                              */
/* ---------------------------------------------------------------------- */
void oracle_filter_taps(double b0[2], double b1[2], double a0[2], double a1[2])
{
    const double s = b00();
    b0[0] = s;  b0[1] = s;
    b1[0] = s;  b1[1] = -s;
    a0[0] = s;  a0[1] = s;
    a1[0] = -s; a1[1] = s;
}

/* Direct analysis level: full-rate convolution with b0 and b1 over every  */
/* input sample (the outputs the decimator throws away are computed too),  */
/* then keep one phase.  With pairs aligned at even indices the kept phase */
/* is the odd one: y[2m+1] = h[0] x[2m+1] + h[1] x[2m].                    */
static void direct_analysis_level(const double* in, double* out, int64_t n,
                                  double* y0, double* y1)
{
    double b0[2], b1[2], a0[2], a1[2];
    oracle_filter_taps(b0, b1, a0, a1);
    for (int64_t k = 0; k < n; ++k) {
        const double cur = in[k];
        const double prev = k > 0 ? in[k - 1] : 0.0;
        y0[k] = b0[0] * cur + b0[1] * prev;
        y1[k] = b1[0] * cur + b1[1] * prev;
    }
    const int64_t pairs = n / 2;
    const int64_t na = n - pairs;
    for (int64_t m = 0; m < pairs; ++m) {    /* decimate: keep odd phase */
        out[m] = y0[2 * m + 1];
        out[na + m] = y1[2 * m + 1];
    }
    if (n & 1) out[pairs] = in[n - 1];
}

/* Direct synthesis level (Eq. (13)): up-sample both channels by 2, filter */
/* with a0 and a1 at the full rate, add.                                   */
static void direct_synthesis_level(const double* in, double* out, int64_t n,
                                   double* u0, double* u1)
{
    double b0[2], b1[2], a0[2], a1[2];
    oracle_filter_taps(b0, b1, a0, a1);
    const int64_t pairs = n / 2;
    const int64_t na = n - pairs;
    const int64_t len = 2 * pairs;
    for (int64_t k = 0; k < len; ++k) { u0[k] = 0.0; u1[k] = 0.0; }
    for (int64_t m = 0; m < pairs; ++m) {    /* up-sample */
        u0[2 * m] = in[m];
        u1[2 * m] = in[na + m];
    }
    for (int64_t k = 0; k < len; ++k) {
        const double p0 = k > 0 ? u0[k - 1] : 0.0;
        const double p1 = k > 0 ? u1[k - 1] : 0.0;
        out[k] = a0[0] * u0[k] + a0[1] * p0 + a1[0] * u1[k] + a1[1] * p1;
    }
    if (n & 1) out[n - 1] = in[pairs];
}

/* ---------------------------------------------------------------------- */
/* Multi-level 1D (dyadic recursion on the approximation).                 */
/* ---------------------------------------------------------------------- */
static void fwd_1d_item(const double* x, double* y, int64_t n, int levels,
                        double* tmp)
{
    memcpy(y, x, (size_t)n * sizeof(double));
    int64_t cur = n;
    for (int j = 1; j <= levels; ++j) {
        memcpy(tmp, y, (size_t)cur * sizeof(double));
        fast_analysis_level(tmp, 1, y, 1, cur);
        cur = (cur + 1) / 2;
    }
}

static void inv_1d_item(const double* y, double* x, int64_t n, int levels,
                        double* tmp)
{
    /* region length before level j: len[j-1]; len[0] = n */
    int64_t len[64];
    len[0] = n;
    for (int j = 1; j <= levels; ++j) len[j] = (len[j - 1] + 1) / 2;
    memcpy(x, y, (size_t)n * sizeof(double));
    for (int j = levels; j >= 1; --j) {
        const int64_t cur = len[j - 1];
        memcpy(tmp, x, (size_t)cur * sizeof(double));
        fast_synthesis_level(tmp, 1, x, 1, cur);
    }
}

void oracle_fwd_1d(const double* x, double* y, int64_t n, int32_t levels,
                   int64_t batch)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < batch; ++b) {
        double* tmp = (double*)malloc((size_t)n * sizeof(double));
        fwd_1d_item(x + b * n, y + b * n, n, levels, tmp);
        free(tmp);
    }
}

void oracle_inv_1d(const double* y, double* x, int64_t n, int32_t levels,
                   int64_t batch)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < batch; ++b) {
        double* tmp = (double*)malloc((size_t)n * sizeof(double));
        inv_1d_item(y + b * n, x + b * n, n, levels, tmp);
        free(tmp);
    }
}

/* Direct-structure multi-level 1D: same recursion, direct bank per level. */
void oracle_direct_fwd_1d(const double* x, double* y, int64_t n,
                          int32_t levels, int64_t batch)
{
    for (int64_t b = 0; b < batch; ++b) {
        double* tmp = (double*)malloc((size_t)n * sizeof(double));
        double* y0 = (double*)malloc((size_t)n * sizeof(double));
        double* y1 = (double*)malloc((size_t)n * sizeof(double));
        double* yb = y + b * n;
        memcpy(yb, x + b * n, (size_t)n * sizeof(double));
        int64_t cur = n;
        for (int j = 1; j <= levels; ++j) {
            memcpy(tmp, yb, (size_t)cur * sizeof(double));
            direct_analysis_level(tmp, yb, cur, y0, y1);
            cur = (cur + 1) / 2;
        }
        free(tmp); free(y0); free(y1);
    }
}

void oracle_direct_inv_1d(const double* y, double* x, int64_t n,
                          int32_t levels, int64_t batch)
{
    for (int64_t b = 0; b < batch; ++b) {
        double* tmp = (double*)malloc((size_t)n * sizeof(double));
        double* u0 = (double*)malloc((size_t)n * sizeof(double));
        double* u1 = (double*)malloc((size_t)n * sizeof(double));
        double* xb = x + b * n;
        int64_t len[64];
        len[0] = n;
        for (int j = 1; j <= levels; ++j) len[j] = (len[j - 1] + 1) / 2;
        memcpy(xb, y + b * n, (size_t)n * sizeof(double));
        for (int j = levels; j >= 1; --j) {
            const int64_t cur = len[j - 1];
            memcpy(tmp, xb, (size_t)cur * sizeof(double));
            direct_synthesis_level(tmp, xb, cur, u0, u1);
        }
        free(tmp); free(u0); free(u1);
    }
}

/* ---------------------------------------------------------------------- */
/* Separable 2D: per level, a 1D level along every row of the current LL   */
/* region (width axis), then along every column (height axis).            */
/* ---------------------------------------------------------------------- */
static void fwd_2d_item(const double* x, double* y, int64_t h, int64_t w,
                        int levels)
{
    memcpy(y, x, (size_t)(h * w) * sizeof(double));
    int64_t ch = h, cw = w;
    for (int j = 1; j <= levels; ++j) {
#pragma omp parallel for schedule(static)
        for (int64_t r = 0; r < ch; ++r) {            /* rows (width)   */
            double* tmp = (double*)malloc((size_t)cw * sizeof(double));
            memcpy(tmp, y + r * w, (size_t)cw * sizeof(double));
            fast_analysis_level(tmp, 1, y + r * w, 1, cw);
            free(tmp);
        }
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < cw; ++c) {            /* columns (height) */
            double* tmp = (double*)malloc((size_t)ch * sizeof(double));
            for (int64_t r = 0; r < ch; ++r) tmp[r] = y[r * w + c];
            fast_analysis_level(tmp, 1, y + c, w, ch);
            free(tmp);
        }
        ch = (ch + 1) / 2;
        cw = (cw + 1) / 2;
    }
}

static void inv_2d_item(const double* y, double* x, int64_t h, int64_t w,
                        int levels)
{
    int64_t lh[64], lw[64];
    lh[0] = h; lw[0] = w;
    for (int j = 1; j <= levels; ++j) {
        lh[j] = (lh[j - 1] + 1) / 2;
        lw[j] = (lw[j - 1] + 1) / 2;
    }
    memcpy(x, y, (size_t)(h * w) * sizeof(double));
    for (int j = levels; j >= 1; --j) {
        const int64_t ch = lh[j - 1], cw = lw[j - 1];
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < cw; ++c) {            /* columns first  */
            double* tmp = (double*)malloc((size_t)ch * sizeof(double));
            for (int64_t r = 0; r < ch; ++r) tmp[r] = x[r * w + c];
            fast_synthesis_level(tmp, 1, x + c, w, ch);
            free(tmp);
        }
#pragma omp parallel for schedule(static)
        for (int64_t r = 0; r < ch; ++r) {            /* then rows      */
            double* tmp = (double*)malloc((size_t)cw * sizeof(double));
            memcpy(tmp, x + r * w, (size_t)cw * sizeof(double));
            fast_synthesis_level(tmp, 1, x + r * w, 1, cw);
            free(tmp);
        }
    }
}

void oracle_fwd_2d(const double* x, double* y, int64_t h, int64_t w,
                   int32_t levels, int64_t batch)
{
    for (int64_t b = 0; b < batch; ++b)
        fwd_2d_item(x + b * h * w, y + b * h * w, h, w, levels);
}

void oracle_inv_2d(const double* y, double* x, int64_t h, int64_t w,
                   int32_t levels, int64_t batch)
{
    for (int64_t b = 0; b < batch; ++b)
        inv_2d_item(y + b * h * w, x + b * h * w, h, w, levels);
}

/* ---------------------------------------------------------------------- */
/* Separable 3D (volumes): per level, a 1D level along every x line (width)  */
/* of the current LLL region, then along every y line (height), then along */
/* every z line (depth); the next level works on the LLL octant            */
/* [0, ceil(d/2)) x [0, ceil(h/2)) x [0, ceil(w/2)).  The synthesis runs z, */
/* y, x per level, levels L..1.  Layout [batch][d][h][w].                  */
/* ---------------------------------------------------------------------- */
static void lines_3d(double* v, int64_t h, int64_t w, int64_t cd, int64_t ch,
                     int64_t cw, int axis, int inverse)
{
    /* axis 0: x lines (length cw), 1: y lines (ch), 2: z lines (cd) */
    const int64_t len = axis == 0 ? cw : (axis == 1 ? ch : cd);
    const int64_t stride = axis == 0 ? 1 : (axis == 1 ? w : h * w);
    const int64_t na = axis == 0 ? cd * ch : (axis == 1 ? cd * cw : ch * cw);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < na; ++q) {
        int64_t base;
        if (axis == 0)      base = (q / ch) * h * w + (q % ch) * w;          /* (z, y) */
        else if (axis == 1) base = (q / cw) * h * w + (q % cw);              /* (z, x) */
        else                base = (q / cw) * w + (q % cw);                  /* (y, x) */
        double* tmp = (double*)malloc((size_t)len * sizeof(double));
        for (int64_t k = 0; k < len; ++k) tmp[k] = v[base + k * stride];
        if (inverse) fast_synthesis_level(tmp, 1, v + base, stride, len);
        else         fast_analysis_level(tmp, 1, v + base, stride, len);
        free(tmp);
    }
}

void oracle_fwd_3d(const double* x, double* y, int64_t d, int64_t h, int64_t w,
                   int32_t levels, int64_t batch)
{
    for (int64_t b = 0; b < batch; ++b) {
        double* v = y + b * d * h * w;
        memcpy(v, x + b * d * h * w, (size_t)(d * h * w) * sizeof(double));
        int64_t cd = d, ch = h, cw = w;
        for (int j = 1; j <= levels; ++j) {
            lines_3d(v, h, w, cd, ch, cw, 0, 0);
            lines_3d(v, h, w, cd, ch, cw, 1, 0);
            lines_3d(v, h, w, cd, ch, cw, 2, 0);
            cd = (cd + 1) / 2;
            ch = (ch + 1) / 2;
            cw = (cw + 1) / 2;
        }
    }
}

void oracle_inv_3d(const double* y, double* x, int64_t d, int64_t h, int64_t w,
                   int32_t levels, int64_t batch)
{
    int64_t ld[64], lh[64], lw[64];
    ld[0] = d; lh[0] = h; lw[0] = w;
    for (int j = 1; j <= levels; ++j) {
        ld[j] = (ld[j - 1] + 1) / 2;
        lh[j] = (lh[j - 1] + 1) / 2;
        lw[j] = (lw[j - 1] + 1) / 2;
    }
    for (int64_t b = 0; b < batch; ++b) {
        double* v = x + b * d * h * w;
        memcpy(v, y + b * d * h * w, (size_t)(d * h * w) * sizeof(double));
        for (int j = levels; j >= 1; --j) {
            lines_3d(v, h, w, ld[j - 1], lh[j - 1], lw[j - 1], 2, 1);
            lines_3d(v, h, w, ld[j - 1], lh[j - 1], lw[j - 1], 1, 1);
            lines_3d(v, h, w, ld[j - 1], lh[j - 1], lw[j - 1], 0, 1);
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Shrinkage of the detail coefficients between analysis and synthesis.   */
/* The paper's applications (Sec. I: compression and analysis of signals  */
/* and images; Sec. VI: biosignals and medical images) decompose, act on   */
/* the coefficients and reconstruct.  Here the action is thresholding of   */
/* every detail coefficient of level j with threshold thr[j-1]:            */
/*   mode 0 (hard): keep d when |d| > t, else 0;                           */
/*   mode 1 (soft): sign(d) * max(|d| - t, 0).                             */
/* The approximation a_L (LL_L) is left unchanged.                          */
/* ---------------------------------------------------------------------- */
static double shrink_value(double d, int mode, double t)
{
    if (mode == 0) return fabs(d) > t ? d : 0.0;
    const double m = fabs(d) - t;
    if (m <= 0.0) return 0.0;
    return d > 0.0 ? m : -m;
}

void oracle_shrink_1d(const double* x, double* y, int64_t n, int32_t levels,
                      int64_t batch, int32_t mode, const double* thr)
{
    double* c = (double*)malloc((size_t)n * sizeof(double));
    int64_t len[64];
    len[0] = n;
    for (int j = 1; j <= levels; ++j) len[j] = (len[j - 1] + 1) / 2;
    for (int64_t b = 0; b < batch; ++b) {
        oracle_fwd_1d(x + b * n, c, n, levels, 1);
        for (int j = 1; j <= levels; ++j)            /* d_j = c[len[j], len[j-1]) */
            for (int64_t i = len[j]; i < len[j - 1]; ++i)
                c[i] = shrink_value(c[i], mode, thr[j - 1]);
        oracle_inv_1d(c, y + b * n, n, levels, 1);
    }
    free(c);
}

void oracle_shrink_2d(const double* x, double* y, int64_t h, int64_t w,
                      int32_t levels, int64_t batch, int32_t mode,
                      const double* thr)
{
    double* c = (double*)malloc((size_t)(h * w) * sizeof(double));
    int64_t lh[64], lw[64];
    lh[0] = h; lw[0] = w;
    for (int j = 1; j <= levels; ++j) {
        lh[j] = (lh[j - 1] + 1) / 2;
        lw[j] = (lw[j - 1] + 1) / 2;
    }
    for (int64_t b = 0; b < batch; ++b) {
        fwd_2d_item(x + b * h * w, c, h, w, levels);
        /* level j bands: the level-(j-1) LL region minus the level-j LL region */
        for (int j = 1; j <= levels; ++j)
            for (int64_t r = 0; r < lh[j - 1]; ++r)
                for (int64_t q = 0; q < lw[j - 1]; ++q)
                    if (r >= lh[j] || q >= lw[j])
                        c[r * w + q] = shrink_value(c[r * w + q], mode, thr[j - 1]);
        inv_2d_item(c, y + b * h * w, h, w, levels);
    }
    free(c);
}

/* ---------------------------------------------------------------------- */
/* Sparsity loss of a training step through the 2D transform and its       */
/* gradient:  c = W x (analysis),  loss = sum |details of levels 1..L|     */
/* + 0.5 * sum LL_L^2,  dloss/dc = (sign(details), LL_L) with sign(0) = 0, */
/* grad_x = W^T dloss/dc, and W^T = W^-1 is the synthesis bank (Sec. IV).  */
/* loss: one value per item.                                               */
/* ---------------------------------------------------------------------- */
void oracle_l1_grad_2d(const double* x, double* g, double* loss, int64_t h,
                       int64_t w, int32_t levels, int64_t batch)
{
    double* c = (double*)malloc((size_t)(h * w) * sizeof(double));
    int64_t hL = h, wL = w;                 /* size of LL_L             */
    for (int j = 1; j <= levels; ++j) {
        hL = (hL + 1) / 2;
        wL = (wL + 1) / 2;
    }
    for (int64_t b = 0; b < batch; ++b) {
        fwd_2d_item(x + b * h * w, c, h, w, levels);
        double l = 0.0;
        for (int64_t r = 0; r < h; ++r)
            for (int64_t q = 0; q < w; ++q) {
                double* v = &c[r * w + q];
                if (r < hL && q < wL) {
                    l += 0.5 * *v * *v;                        /* LL_L      */
                } else {
                    l += fabs(*v);                             /* a detail  */
                    *v = *v > 0.0 ? 1.0 : (*v < 0.0 ? -1.0 : 0.0);
                }
            }
        loss[b] = l;
        inv_2d_item(c, g + b * h * w, h, w, levels);
    }
    free(c);
}

/* Number of OpenMP threads the oracle runs with (1 without OpenMP). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
