/*
 * CPU oracle for the complex DFT on separate real and imaginary planes
 * (A. Cariow, "Fast algorithms for complex-valued discrete Fourier transform
 * with separate real and imaginary inputs/outputs", arXiv 2504.07264).
 *
 * TEST INFRASTRUCTURE ONLY.  The product library never links, loads or calls
 * this file.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or constant
 * generator with the GPU library; the two agree only because both follow the
 * paper.
 *
 * What is here, each written plainly, with no blocking or fusion:
 *   - the twiddle blocks omega^(i,q) of Section III (definitions under eq. 6);
 *   - O1: the DFT of eq. (1), written as the real block product of eq. (5),
 *     evaluated directly in O(N^2) FP64, forward and adjoint;
 *   - O2: the decimation-in-time factorisation of eq. (6), applied factor by
 *     factor in FP64 on the two planes;
 *   - O2f: the same factor sequence in FP32 with one fixed operation form per
 *     step, used as the structural mirror for bit-exact checks;
 *   - O3: the decimation-in-frequency factorisation of eq. (9), FP64 and FP32.
 *
 * Conventions (readings of the paper, each pinned by a test):
 *   - N = 2^m.  The paper states m >= 2 (Section III); m = 0 and m = 1 follow
 *     from the same formulas and are accepted here.
 *   - Forward transform with the negative exponent of eq. (1), unnormalised.
 *   - Planes: eq. (5) acts on [xr; xi].  Eq. (6) acts on the interleaved
 *     vector x_2N = [x0r, x0i, x1r, x1i, ...].  Every factor of eq. (6) is
 *     either a permutation of whole pairs, a butterfly between whole pairs or a
 *     2x2 block on one pair, so each factor is applied here to the pair
 *     (xr[k], xi[k]) held in two arrays.
 *   - The leading identity of W^(i) and D^(i) in eq. (6) has order 2^(m-i)
 *     (the worked example of Section III uses this order; the general formula
 *     prints 2^(m-1), which gives the wrong dimension for i > 1).
 *   - omega^(i,q) always follows the formula under eq. (6).  The worked
 *     example's printed omega^(3,3) (eq. 8) repeats omega^(3,1) and is not
 *     used.
 *   - The permutation S_(2^m): output element k is input element rev_m(k)
 *     (0-based indices).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif
#ifndef M_SQRT1_2
#define M_SQRT1_2 0.70710678118654752440
#endif

/* Bit reversal of the m-bit index n (Section III, definition of S_(2^m)). */
static int64_t rev_bits(int64_t n, int m)
{
    int64_t r = 0;
    for (int b = 0; b < m; ++b)
        if ((n >> b) & 1)
            r |= (int64_t)1 << (m - 1 - b);
    return r;
}

int64_t oracle_bit_reverse(int64_t n, int m) { return rev_bits(n, m); }

/*
 * omega^(i,q) = [[cos t, sin t], [-sin t, cos t]], t = 2*pi*q / 2^i
 * (Section III, definitions under eq. 6).  Returned as (cos t, sin t).
 *
 * Values are made exact where the angle is a multiple of pi/4: write
 * 4q = k*2^i + r with the remainder r taken in (-2^i/2, 2^i/2], so that
 * t = (pi/2) * (k + r/2^i).  The local angle phi = (pi/2) * r/2^i lies in
 * [-pi/4, pi/4].  If |phi| = pi/4 both local cos and |sin| are 1/sqrt(2)
 * (the same FP64 number); otherwise they are libm cos and sin of
 * |phi| = (pi*|r|) / (2 * 2^i), with the sign of r given to sin.  The
 * quadrant k (mod 4) then rotates (cos phi, sin phi) by k*pi/2.  So 0 and +-1
 * come out exact and cos = sin at pi/4.  A negative zero is returned as +0.
 */
void oracle_omega_f64(int64_t q, int i, double *c_out, double *s_out)
{
    const int64_t d = (int64_t)1 << i;
    int64_t k = (4 * q) / d;
    int64_t r = (4 * q) % d;
    if (2 * r > d) { /* take the remainder in (-d/2, d/2] */
        k += 1;
        r -= d;
    }
    double cl, sl;
    const int64_t ar = r < 0 ? -r : r;
    if (2 * ar == d) {
        cl = M_SQRT1_2;
        sl = M_SQRT1_2;
    } else {
        const double phi = (M_PI * (double)ar) / (2.0 * (double)d);
        cl = cos(phi);
        sl = sin(phi);
    }
    if (r < 0)
        sl = -sl;
    double c, s;
    switch ((int)(((k % 4) + 4) % 4)) {
    case 0: c = cl;  s = sl;  break;
    case 1: c = -sl; s = cl;  break;
    case 2: c = -cl; s = -sl; break;
    default: c = sl; s = -cl; break;
    }
    *c_out = c + 0.0; /* -0 -> +0 */
    *s_out = s + 0.0;
}

/*
 * Table of all twiddles a transform of length 2^m uses: entry 2^(i-1) + q
 * holds omega^(i,q) for stage i = 1..m and q = 0..2^(i-1)-1.  Entry 0 holds
 * the angle 0.  FP64 and FP32 (round to nearest) versions.
 */
void oracle_twiddle_table_f64(int m, double *c, double *s)
{
    c[0] = 1.0;
    s[0] = 0.0;
    for (int i = 1; i <= m; ++i) {
        const int64_t half = (int64_t)1 << (i - 1);
        for (int64_t q = 0; q < half; ++q)
            oracle_omega_f64(q, i, &c[half + q], &s[half + q]);
    }
}

void oracle_twiddle_table_f32(int m, float *c, float *s)
{
    const int64_t n = (int64_t)1 << m;
    double *cd = (double *)malloc(sizeof(double) * (size_t)(n > 1 ? n : 1));
    double *sd = (double *)malloc(sizeof(double) * (size_t)(n > 1 ? n : 1));
    oracle_twiddle_table_f64(m, cd, sd);
    for (int64_t j = 0; j < n; ++j) {
        c[j] = (float)cd[j] + 0.0f;
        s[j] = (float)sd[j] + 0.0f;
    }
    free(cd);
    free(sd);
}

static int log2_exact(int64_t n)
{
    int m = 0;
    while (((int64_t)1 << m) < n)
        ++m;
    return (((int64_t)1 << m) == n) ? m : -1;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------
 * O1: direct evaluation of eq. (5), E_2N = [[C, S], [-S, C]] with
 * c_{k,n} = cos(2 pi k n / N), s_{k,n} = sin(2 pi k n / N) (eq. 3).
 *   yr_k = sum_n  xr_n c_{k,n} + xi_n s_{k,n}
 *   yi_k = sum_n -xr_n s_{k,n} + xi_n c_{k,n}
 * The product k*n is reduced mod N in integers before the table lookup, so
 * the angle is never large.  Tables are plain libm values, independent of the
 * twiddle rule above.
 * ---------------------------------------------------------------------- */
static void direct_tables(int64_t n, double **c, double **s)
{
    *c = (double *)malloc(sizeof(double) * (size_t)n);
    *s = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t r = 0; r < n; ++r) {
        const double t = 2.0 * M_PI * (double)r / (double)n;
        (*c)[r] = cos(t);
        (*s)[r] = sin(t);
    }
}

int oracle_dft_direct_f64(int64_t n, int64_t batch, const double *xr, const double *xi,
                          double *yr, double *yi, int nthreads)
{
    if (n < 1 || batch < 0)
        return -1;
    double *c, *s;
    direct_tables(n, &c, &s);
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < batch; ++b) {
        const double *ar = xr + b * n, *ai = xi + b * n;
        for (int64_t k = 0; k < n; ++k) {
            double accr = 0.0, acci = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                const int64_t r = (k * j) % n;
                accr += ar[j] * c[r] + ai[j] * s[r];
                acci += -ar[j] * s[r] + ai[j] * c[r];
            }
            yr[b * n + k] = accr;
            yi[b * n + k] = acci;
        }
    }
    free(c);
    free(s);
    return 0;
}

/* O1 at selected output bins k of one row (for sampled checks at full size). */
int oracle_dft_direct_bins_f64(int64_t n, const double *xr, const double *xi, int64_t nk,
                               const int64_t *ks, double *yr, double *yi)
{
    if (n < 1 || nk < 0)
        return -1;
    double *c, *s;
    direct_tables(n, &c, &s);
    for (int64_t t = 0; t < nk; ++t) {
        const int64_t k = ks[t];
        double accr = 0.0, acci = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const int64_t r = (k * j) % n;
            accr += xr[j] * c[r] + xi[j] * s[r];
            acci += -xr[j] * s[r] + xi[j] * c[r];
        }
        yr[t] = accr;
        yi[t] = acci;
    }
    free(c);
    free(s);
    return 0;
}

/*
 * O1 adjoint: the transpose of E_2N of eq. (5).  C and S are symmetric, so
 * E_2N^T = [[C, -S], [S, C]]:
 *   gxr_n = sum_k  gr_k c_{k,n} - gi_k s_{k,n}
 *   gxi_n = sum_k  gr_k s_{k,n} + gi_k c_{k,n}
 * Evaluated directly, not through any identity with the forward transform.
 */
int oracle_adjoint_direct_f64(int64_t n, int64_t batch, const double *gr, const double *gi,
                              double *gxr, double *gxi, int nthreads)
{
    if (n < 1 || batch < 0)
        return -1;
    double *c, *s;
    direct_tables(n, &c, &s);
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < batch; ++b) {
        const double *ar = gr + b * n, *ai = gi + b * n;
        for (int64_t j = 0; j < n; ++j) {
            double accr = 0.0, acci = 0.0;
            for (int64_t k = 0; k < n; ++k) {
                const int64_t r = (k * j) % n;
                accr += ar[k] * c[r] - ai[k] * s[r];
                acci += ar[k] * s[r] + ai[k] * c[r];
            }
            gxr[b * n + j] = accr;
            gxi[b * n + j] = acci;
        }
    }
    free(c);
    free(s);
    return 0;
}

/* ------------------------------------------------------------------------
 * O2: eq. (6), y_2N = W^(m) D^(m) ... W^(1) D^(1) S x_2N, applied right to
 * left on the two planes.
 *   S      : (y_k) = x_(rev_m k) on both planes.
 *   D^(i)  : I_(2^(m-i)) (x) diag(I_(2R), omega^(i,0), ..., omega^(i,R-1)),
 *            R = 2^(i-1): in each block of 2^i complex elements, the element
 *            at offset R + q is multiplied by the 2x2 block omega^(i,q):
 *              (ar, ai) -> (c ar + s ai, -s ar + c ai).
 *   W^(i)  : I_(2^(m-i)) (x) H_2 (x) I_(2^i): in each block of 2^i complex
 *            elements, element q and element R + q become (u + v, u - v),
 *            separately in each plane.
 * ---------------------------------------------------------------------- */
static void dit_row_f64(int m, const double *tc, const double *ts, const double *xr,
                        const double *xi, double *yr, double *yi)
{
    const int64_t n = (int64_t)1 << m;
    for (int64_t k = 0; k < n; ++k) { /* S */
        yr[k] = xr[rev_bits(k, m)];
        yi[k] = xi[rev_bits(k, m)];
    }
    for (int i = 1; i <= m; ++i) {
        const int64_t R = (int64_t)1 << (i - 1);
        for (int64_t base = 0; base < n; base += 2 * R) {
            for (int64_t q = 0; q < R; ++q) {
                const int64_t lo = base + q, up = base + R + q;
                const double c = tc[R + q], s = ts[R + q];
                /* D^(i) on the upper element */
                const double vr = c * yr[up] + s * yi[up];
                const double vi = -s * yr[up] + c * yi[up];
                /* W^(i) between the halves */
                const double ur = yr[lo], ui = yi[lo];
                yr[lo] = ur + vr;
                yi[lo] = ui + vi;
                yr[up] = ur - vr;
                yi[up] = ui - vi;
            }
        }
    }
}

int oracle_split_fft_f64(int64_t n, int64_t batch, const double *xr, const double *xi,
                         double *yr, double *yi, int nthreads)
{
    const int m = log2_exact(n);
    if (m < 0 || batch < 0)
        return -1;
    double *tc = (double *)malloc(sizeof(double) * (size_t)n);
    double *ts = (double *)malloc(sizeof(double) * (size_t)n);
    oracle_twiddle_table_f64(m, tc, ts);
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < batch; ++b)
        dit_row_f64(m, tc, ts, xr + b * n, xi + b * n, yr + b * n, yi + b * n);
    free(tc);
    free(ts);
    return 0;
}

/*
 * O2f: the same factor sequence in FP32.  Every step has one fixed form so
 * that another FP32 evaluation of eq. (6) in the same order can be compared
 * bit for bit:
 *   D^(i):  tr = fmaf(c, ar, s * ai);  ti = fmaf(c, ai, -(s * ar));
 *   W^(i):  u + v and u - v.
 * (c, s) are the FP32 roundings of the FP64 twiddles above.  This file is
 * compiled with floating-point contraction off, so no other fused operation
 * appears.
 */
static void dit_row_f32(int m, const float *tc, const float *ts, const float *xr,
                        const float *xi, float *yr, float *yi)
{
    const int64_t n = (int64_t)1 << m;
    for (int64_t k = 0; k < n; ++k) {
        yr[k] = xr[rev_bits(k, m)];
        yi[k] = xi[rev_bits(k, m)];
    }
    for (int i = 1; i <= m; ++i) {
        const int64_t R = (int64_t)1 << (i - 1);
        for (int64_t base = 0; base < n; base += 2 * R) {
            for (int64_t q = 0; q < R; ++q) {
                const int64_t lo = base + q, up = base + R + q;
                const float c = tc[R + q], s = ts[R + q];
                const float ar = yr[up], ai = yi[up];
                const float vr = fmaf(c, ar, s * ai);
                const float vi = fmaf(c, ai, -(s * ar));
                const float ur = yr[lo], ui = yi[lo];
                yr[lo] = ur + vr;
                yi[lo] = ui + vi;
                yr[up] = ur - vr;
                yi[up] = ui - vi;
            }
        }
    }
}

int oracle_split_fft_f32(int64_t n, int64_t batch, const float *xr, const float *xi,
                         float *yr, float *yi, int nthreads)
{
    const int m = log2_exact(n);
    if (m < 0 || batch < 0)
        return -1;
    float *tc = (float *)malloc(sizeof(float) * (size_t)n);
    float *ts = (float *)malloc(sizeof(float) * (size_t)n);
    oracle_twiddle_table_f32(m, tc, ts);
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < batch; ++b)
        dit_row_f32(m, tc, ts, xr + b * n, xi + b * n, yr + b * n, yi + b * n);
    free(tc);
    free(ts);
    return 0;
}

/* ------------------------------------------------------------------------
 * O3: eq. (9), y_2N = S D^(1) W^(1) ... D^(m) W^(m) x_2N, applied right to
 * left: for i = m down to 1, first W^(i) (butterfly between the halves of
 * each 2^i block), then D^(i) (rotate the upper half by omega^(i,q)); the
 * permutation S comes last.
 * ---------------------------------------------------------------------- */
static void dif_row_f64(int m, const double *tc, const double *ts, const double *xr,
                        const double *xi, double *yr, double *yi, double *wr, double *wi)
{
    const int64_t n = (int64_t)1 << m;
    memcpy(wr, xr, sizeof(double) * (size_t)n);
    memcpy(wi, xi, sizeof(double) * (size_t)n);
    for (int i = m; i >= 1; --i) {
        const int64_t R = (int64_t)1 << (i - 1);
        for (int64_t base = 0; base < n; base += 2 * R) {
            for (int64_t q = 0; q < R; ++q) {
                const int64_t lo = base + q, up = base + R + q;
                const double ur = wr[lo], ui = wi[lo], vr = wr[up], vi = wi[up];
                wr[lo] = ur + vr; /* W^(i) */
                wi[lo] = ui + vi;
                const double dr = ur - vr, di = ui - vi;
                const double c = tc[R + q], s = ts[R + q];
                wr[up] = c * dr + s * di; /* D^(i) */
                wi[up] = -s * dr + c * di;
            }
        }
    }
    for (int64_t k = 0; k < n; ++k) { /* S */
        yr[k] = wr[rev_bits(k, m)];
        yi[k] = wi[rev_bits(k, m)];
    }
}

int oracle_split_fft_dif_f64(int64_t n, int64_t batch, const double *xr, const double *xi,
                             double *yr, double *yi, int nthreads)
{
    const int m = log2_exact(n);
    if (m < 0 || batch < 0)
        return -1;
    double *tc = (double *)malloc(sizeof(double) * (size_t)n);
    double *ts = (double *)malloc(sizeof(double) * (size_t)n);
    oracle_twiddle_table_f64(m, tc, ts);
    set_threads(nthreads);
#pragma omp parallel
    {
        double *wr = (double *)malloc(sizeof(double) * (size_t)n);
        double *wi = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
        for (int64_t b = 0; b < batch; ++b)
            dif_row_f64(m, tc, ts, xr + b * n, xi + b * n, yr + b * n, yi + b * n, wr, wi);
        free(wr);
        free(wi);
    }
    free(tc);
    free(ts);
    return 0;
}

/* O3 in FP32 with the fixed forms of O2f (rotation, then u + v / u - v). */
static void dif_row_f32(int m, const float *tc, const float *ts, const float *xr,
                        const float *xi, float *yr, float *yi, float *wr, float *wi)
{
    const int64_t n = (int64_t)1 << m;
    memcpy(wr, xr, sizeof(float) * (size_t)n);
    memcpy(wi, xi, sizeof(float) * (size_t)n);
    for (int i = m; i >= 1; --i) {
        const int64_t R = (int64_t)1 << (i - 1);
        for (int64_t base = 0; base < n; base += 2 * R) {
            for (int64_t q = 0; q < R; ++q) {
                const int64_t lo = base + q, up = base + R + q;
                const float ur = wr[lo], ui = wi[lo], vr = wr[up], vi = wi[up];
                wr[lo] = ur + vr;
                wi[lo] = ui + vi;
                const float dr = ur - vr, di = ui - vi;
                const float c = tc[R + q], s = ts[R + q];
                wr[up] = fmaf(c, dr, s * di);
                wi[up] = fmaf(c, di, -(s * dr));
            }
        }
    }
    for (int64_t k = 0; k < n; ++k) {
        yr[k] = wr[rev_bits(k, m)];
        yi[k] = wi[rev_bits(k, m)];
    }
}

int oracle_split_fft_dif_f32(int64_t n, int64_t batch, const float *xr, const float *xi,
                             float *yr, float *yi, int nthreads)
{
    const int m = log2_exact(n);
    if (m < 0 || batch < 0)
        return -1;
    float *tc = (float *)malloc(sizeof(float) * (size_t)n);
    float *ts = (float *)malloc(sizeof(float) * (size_t)n);
    oracle_twiddle_table_f32(m, tc, ts);
    set_threads(nthreads);
#pragma omp parallel
    {
        float *wr = (float *)malloc(sizeof(float) * (size_t)n);
        float *wi = (float *)malloc(sizeof(float) * (size_t)n);
#pragma omp for schedule(static)
        for (int64_t b = 0; b < batch; ++b)
            dif_row_f32(m, tc, ts, xr + b * n, xi + b * n, yr + b * n, yi + b * n, wr, wi);
        free(wr);
        free(wi);
    }
    free(tc);
    free(ts);
    return 0;
}
