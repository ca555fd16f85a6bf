/*
 * dd_oracle.c -- plain FP64 CPU evaluation of the alpha-dense DFT.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the GPU path.
 *
 * What it computes (paper, Section 2):
 *   The alpha-dense DFT, eq. (7) first line, on the frequency grid of eq. (6)
 *   (nu_m = m / (alpha*T), m = 0 .. alpha*N-1), with the forward scaling T/N
 *   of the sampled transform, eq. (2):
 *
 *       X_m = (T/N) * sum_{n=0}^{N-1} x_n * exp(-2*pi*i * m*n / (alpha*N))
 *
 *   The sign convention is the one the paper fixes for W (Section 3,
 *   W_N^{mn} = exp(-2 pi i mn / N)).  This is the plain definition, summed
 *   directly, O(alpha*N) work per output bin; no FFT structure is used here.
 *
 * Arithmetic:
 *   - inputs are the exact stored samples promoted to double (real input has
 *     a zero imaginary part);
 *   - the phase exponent is reduced exactly in integers, q = (m*n) mod M with
 *     M = alpha*N, by stepping q <- q + m (mod M) along n; m < M, so one
 *     conditional subtraction keeps q in [0, M);
 *   - theta = 2*pi*q/M in double, cos/sin from libm;
 *   - when M <= ORACLE_TABLE_MAX the values cos/sin(2 pi q / M), q < M, are
 *     computed once with the same libm calls and looked up (a cache of the
 *     same numbers, not a different formula);
 *   - the sum runs sequentially over n in the paper's order, in double.
 *
 * Bins are independent; they are spread over OpenMP threads.
 *
 * The "mutation" argument exists only so that the test suite can plant a
 * known mistake in this oracle and show that its pins catch it.  0 means the
 * correct definition above; any other value is a deliberately wrong variant
 * (see the switch below) and must never be used to produce expected values.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_TABLE_MAX (1LL << 22)

static const double TWO_PI = 6.283185307179586476925286766559;

int dd_oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Returns 0 on success, -1 on invalid arguments, -2 on allocation failure. */
int dd_oracle_bins_mut(const double *xr, const double *xi, int64_t N,
                       int64_t alpha, double T, const int64_t *bins,
                       int64_t nbins, double *outr, double *outi,
                       int mutation)
{
    if (N < 1 || alpha < 1 || nbins < 0 || !xr || !xi || (nbins && (!bins || !outr || !outi)))
        return -1;
    const int64_t M = alpha * N;
    for (int64_t b = 0; b < nbins; ++b)
        if (bins[b] < 0 || bins[b] >= M) return -1;

    /* mutation 5: forget alpha (use the conventional N-point grid) */
    const int64_t Meff = (mutation == 5) ? N : M;

    double *tc = NULL, *ts = NULL;
    if (Meff <= ORACLE_TABLE_MAX) {
        tc = (double *)malloc(sizeof(double) * (size_t)Meff);
        ts = (double *)malloc(sizeof(double) * (size_t)Meff);
        if (!tc || !ts) { free(tc); free(ts); return -2; }
        #pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < Meff; ++q) {
            double th = TWO_PI * ((double)q / (double)Meff);
            tc[q] = cos(th);
            ts[q] = sin(th);
        }
    }

    /* eq. (2): forward factor T/N (mutation 4 drops T) */
    const double scale = (mutation == 4) ? 1.0 / (double)N : T / (double)N;
    const int64_t nlast = (mutation == 2) ? N - 1 : N;   /* mutation 2: drop the last term */

    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < nbins; ++b) {
        const int64_t m = bins[b] % Meff;
        double ar = 0.0, ai = 0.0;
        uint64_t q = 0;                           /* q = (m*n) mod Meff */
        for (int64_t n = 0; n < nlast; ++n) {
            double c, s;
            if (tc) { c = tc[q]; s = ts[q]; }
            else {
                double th = TWO_PI * ((double)q / (double)Meff);
                c = cos(th); s = sin(th);
            }
            if (mutation == 1) s = -s;            /* mutation 1: wrong sign of the exponent */
            int64_t src = n;
            if (mutation == 3) src = (n + 1) % N; /* mutation 3: off-by-one sample index */
            double pr = xr[src], pi = xi[src];
            if (mutation == 6) { double t = pr; pr = pi; pi = t; } /* mutation 6: re/im swapped */
            /* x_n * (cos th - i sin th) */
            ar += pr * c + pi * s;
            ai += pi * c - pr * s;
            q += (uint64_t)m;
            if (q >= (uint64_t)Meff) q -= (uint64_t)Meff;
        }
        outr[b] = scale * ar;
        outi[b] = scale * ai;
    }
    free(tc);
    free(ts);
    return 0;
}

/* The inverse alpha-transform (the reading of eq. (7), second line, with the
 * 1/(alpha T) factor that makes it undo the forward transform of eq. (2)):
 *     x_n = (1/(alpha T)) * sum_{m < alpha N} X_m * exp(+2 pi i m n / (alpha N)),
 * evaluated at the requested samples n (0 <= n < alpha N; the transform of a
 * forward spectrum vanishes for n >= N).  Direct FP64 sum, exact integer
 * phase q = (m n) mod alpha N.  Mutations (for the tests that check the pins
 * reject a wrong inverse): 1 wrong exponent sign, 2 factor 1/T (alpha
 * dropped), 3 sum over m < N only, 4 spectrum index off by one.
 * Returns 0 on success, -1 on invalid arguments, -2 on allocation failure. */
int dd_oracle_inv_mut(const double *Xr, const double *Xi, int64_t N, int64_t alpha,
                      double T, const int64_t *samples, int64_t ns, double *outr,
                      double *outi, int mutation)
{
    if (N < 1 || alpha < 1 || ns < 0 || !Xr || !Xi || (ns && (!samples || !outr || !outi)))
        return -1;
    const int64_t M = alpha * N;
    for (int64_t b = 0; b < ns; ++b)
        if (samples[b] < 0 || samples[b] >= M) return -1;
    double *tc = NULL, *ts = NULL;
    if (M <= ORACLE_TABLE_MAX) {
        tc = (double *)malloc(sizeof(double) * (size_t)M);
        ts = (double *)malloc(sizeof(double) * (size_t)M);
        if (!tc || !ts) { free(tc); free(ts); return -2; }
        #pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < M; ++q) {
            double th = TWO_PI * ((double)q / (double)M);
            tc[q] = cos(th);
            ts[q] = sin(th);
        }
    }
    const double scale = (mutation == 2) ? 1.0 / T : 1.0 / ((double)alpha * T);
    const int64_t mlast = (mutation == 3) ? N : M;

    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < ns; ++b) {
        const int64_t n = samples[b];
        double ar = 0.0, ai = 0.0;
        uint64_t q = 0;                           /* q = (m*n) mod M */
        for (int64_t m = 0; m < mlast; ++m) {
            double c, s;
            if (tc) { c = tc[q]; s = ts[q]; }
            else {
                double th = TWO_PI * ((double)q / (double)M);
                c = cos(th); s = sin(th);
            }
            if (mutation == 1) s = -s;
            const int64_t src = (mutation == 4) ? (m + 1) % M : m;
            const double pr = Xr[src], pi = Xi[src];
            /* X_m * (cos th + i sin th) */
            ar += pr * c - pi * s;
            ai += pi * c + pr * s;
            q += (uint64_t)n;
            if (q >= (uint64_t)M) q -= (uint64_t)M;
        }
        outr[b] = scale * ar;
        outi[b] = scale * ai;
    }
    free(tc);
    free(ts);
    return 0;
}

int dd_oracle_bins(const double *xr, const double *xi, int64_t N, int64_t alpha,
                   double T, const int64_t *bins, int64_t nbins, double *outr,
                   double *outi)
{
    return dd_oracle_bins_mut(xr, xi, N, alpha, T, bins, nbins, outr, outi, 0);
}
