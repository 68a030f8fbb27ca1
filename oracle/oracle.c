/*
 * FX-correlator oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * A plain, slow, obviously-correct CPU statement of what the correlator hot
 * path computes (Wang & Harris, "Scaling Radio Astronomy Signal Correlation on
 * Heterogeneous Supercomputers ...", Exp. Astron. 2013):
 *
 *   - F-engine, Section 2 Eq. 1:  S[k] = sum_{n=0}^{C-1} s[n] exp(-j 2 pi k n / C),
 *     a direct DFT in float64, applied to consecutive non-overlapping blocks of
 *     C samples (block a uses samples [aC, (a+1)C)), natural channel order, no
 *     normalisation, no window.  The real-input form (Section 5: 8-bit real
 *     samples, transform length 256) takes blocks of 2C real samples and keeps
 *     channels 0..C of their length-2C DFT.
 *   - X-engine, Section 2 Eq. 2:  C_ij[k] = sum_{a=0}^{A-1} conj(S_{a,i}[k]) S_{a,j}[k],
 *     conjugate on the first index, summed (not averaged) over A spectra, over
 *     the triangle of non-redundant pairs including the autos (Section 4).
 *     float64 accumulation for float inputs, int64 for 8-bit integer inputs
 *     (Section 5: inputs packed in 8-bit integers).
 *   - Requantisers (the reduced-precision forms of the spectra): int8 with
 *     round-half-to-even and a symmetric clamp to +-127; IEEE binary16 and the
 *     OCP FP8 E4M3 format, both round-half-to-even with saturation to the
 *     largest finite value.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * call this code.  It shares no source with the GPU library.
 *
 * Every routine here is pinned in the CPU test suite against something other
 * than itself: library special cases, closed forms, invariants and brute force.
 *
 * Visibility triangle index (lower triangle, autos included):
 *   row i in [0,N), column j in [0,i], b(i,j) = i(i+1)/2 + j.
 *
 * Complex numbers are stored as interleaved (re, im) pairs throughout.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* F-engine: Eq. 1                                                            */
/* ------------------------------------------------------------------------- */

/*
 * Direct DFT of every block a in [0, n_spectra) of every input p in
 * [0, n_inputs), evaluated only at the channels listed in chans[0..n_chans).
 *
 *   volts : complex64 [n_inputs][ld] (float re, im interleaved); block a of
 *           input p is volts[p][a*C .. a*C + C).
 *   S     : complex128 [n_spectra][n_inputs][n_chans] output,
 *           S[a][p][c] = sum_n s_p[aC + n] * exp(-j 2 pi chans[c] n / C).
 *
 * The exponent's argument is reduced exactly in integers, m = (k n) mod C,
 * before the float64 cos/sin of 2 pi m / C, so the twiddle error does not grow
 * with k n.  The table w[m] = exp(-j 2 pi m / C) holds those C values.
 */
void oracle_fengine(const float *volts, int64_t ld, int n_inputs, int C,
                    int n_spectra, const int *chans, int n_chans, double *S)
{
    const double two_pi = 6.283185307179586476925286766559;
    double *w = (double *)malloc(sizeof(double) * 2 * (size_t)C);
    for (int m = 0; m < C; ++m) {
        w[2 * m + 0] = cos(two_pi * (double)m / (double)C);
        w[2 * m + 1] = -sin(two_pi * (double)m / (double)C);
    }
    const int64_t total = (int64_t)n_spectra * n_inputs;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t ap = 0; ap < total; ++ap) {
        const int a = (int)(ap / n_inputs);
        const int p = (int)(ap % n_inputs);
        const float *s = volts + 2 * ((int64_t)p * ld + (int64_t)a * C);
        for (int c = 0; c < n_chans; ++c) {
            const int k = chans[c];
            double re = 0.0, im = 0.0;
            int m = 0; /* m = (k n) mod C, advanced by k each step */
            for (int n = 0; n < C; ++n) {
                const double sr = (double)s[2 * n], si = (double)s[2 * n + 1];
                const double wr = w[2 * m], wi = w[2 * m + 1];
                re += sr * wr - si * wi;
                im += sr * wi + si * wr;
                m += k;
                if (m >= C)
                    m -= C;
            }
            double *o = S + 2 * ((ap) * n_chans + c);
            o[0] = re;
            o[1] = im;
        }
    }
    free(w);
}

/*
 * Real-input form of Eq. 1 (Section 5: the test streams are 8-bit real
 * samples and the transform length is 256).  Block a of input p is the 2C
 * real samples x_p[a*2C .. a*2C + 2C); its spectrum is the DFT of length 2C,
 *
 *   X[a][p][c] = sum_{n=0}^{2C-1} x_p[a*2C + n] * exp(-j 2 pi k n / (2C)),
 *   k = chans[c] in [0, C]  (C itself is the Nyquist channel),
 *
 * evaluated directly in float64 with the argument reduced exactly,
 * m = (k n) mod 2C, as in oracle_fengine.
 *   x : int8 [n_inputs][ld] real samples.
 *   S : complex128 [n_spectra][n_inputs][n_chans] output.
 */
void oracle_fengine_real8(const int8_t *x, int64_t ld, int n_inputs, int C, int n_spectra,
                          const int *chans, int n_chans, double *S)
{
    const double two_pi = 6.283185307179586476925286766559;
    const int L = 2 * C;
    double *w = (double *)malloc(sizeof(double) * 2 * (size_t)L);
    for (int m = 0; m < L; ++m) {
        w[2 * m + 0] = cos(two_pi * (double)m / (double)L);
        w[2 * m + 1] = -sin(two_pi * (double)m / (double)L);
    }
    const int64_t total = (int64_t)n_spectra * n_inputs;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t ap = 0; ap < total; ++ap) {
        const int a = (int)(ap / n_inputs);
        const int p = (int)(ap % n_inputs);
        const int8_t *s = x + (int64_t)p * ld + (int64_t)a * L;
        for (int c = 0; c < n_chans; ++c) {
            const int k = chans[c];
            double re = 0.0, im = 0.0;
            int m = 0; /* m = (k n) mod 2C */
            for (int n = 0; n < L; ++n) {
                const double v = (double)s[n];
                re += v * w[2 * m];
                im += v * w[2 * m + 1];
                m += k;
                if (m >= L)
                    m -= L;
            }
            double *o = S + 2 * (ap * n_chans + c);
            o[0] = re;
            o[1] = im;
        }
    }
    free(w);
}

/* ------------------------------------------------------------------------- */
/* X-engine: Eq. 2 over the triangle of non-redundant pairs                   */
/* ------------------------------------------------------------------------- */

/*
 * float64 correlation.
 *   S : complex128 [A][N][K]  (spectrum a, input i, channel k)
 *   V : complex128 [K][N(N+1)/2] output, V[k][b(i,j)] = sum_a conj(S[a][i][k]) S[a][j][k]
 *       for j <= i.  The auto terms use re^2 + im^2, so their imaginary part is 0.
 */
void oracle_xengine_f64(const double *S, int A, int N, int K, double *V)
{
    const int64_t B = (int64_t)N * (N + 1) / 2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < K; ++k) {
        /* Gather channel k into X[i][a] so the sum over a walks memory in order. */
        double *X = (double *)malloc(sizeof(double) * 2 * (size_t)N * (size_t)A);
        for (int a = 0; a < A; ++a)
            for (int i = 0; i < N; ++i) {
                const double *src = S + 2 * (((int64_t)a * N + i) * K + k);
                X[2 * ((int64_t)i * A + a) + 0] = src[0];
                X[2 * ((int64_t)i * A + a) + 1] = src[1];
            }
        for (int i = 0; i < N; ++i) {
            const double *xi = X + 2 * (int64_t)i * A;
            for (int j = 0; j <= i; ++j) {
                const double *xj = X + 2 * (int64_t)j * A;
                double re = 0.0, im = 0.0;
                if (i == j) {
                    for (int a = 0; a < A; ++a)
                        re += xi[2 * a] * xi[2 * a] + xi[2 * a + 1] * xi[2 * a + 1];
                } else {
                    for (int a = 0; a < A; ++a) {
                        /* conj(x_i) * x_j */
                        re += xi[2 * a] * xj[2 * a] + xi[2 * a + 1] * xj[2 * a + 1];
                        im += xi[2 * a] * xj[2 * a + 1] - xi[2 * a + 1] * xj[2 * a];
                    }
                }
                double *o = V + 2 * ((int64_t)k * B + (int64_t)i * (i + 1) / 2 + j);
                o[0] = re;
                o[1] = im;
            }
        }
        free(X);
    }
}

/*
 * Exact integer correlation of 8-bit spectra.
 *   S : int8 [A][N][K][2]  (re, im)
 *   V : int64 [K][N(N+1)/2][2] output, same definition as above, exact.
 */
void oracle_xengine_i8(const int8_t *S, int A, int N, int K, int64_t *V)
{
    const int64_t B = (int64_t)N * (N + 1) / 2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < K; ++k) {
        int32_t *X = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)N * (size_t)A);
        for (int a = 0; a < A; ++a)
            for (int i = 0; i < N; ++i) {
                const int8_t *src = S + 2 * (((int64_t)a * N + i) * K + k);
                X[2 * ((int64_t)i * A + a) + 0] = src[0];
                X[2 * ((int64_t)i * A + a) + 1] = src[1];
            }
        for (int i = 0; i < N; ++i) {
            const int32_t *xi = X + 2 * (int64_t)i * A;
            for (int j = 0; j <= i; ++j) {
                const int32_t *xj = X + 2 * (int64_t)j * A;
                int64_t re = 0, im = 0;
                for (int a = 0; a < A; ++a) {
                    re += (int64_t)xi[2 * a] * xj[2 * a] + (int64_t)xi[2 * a + 1] * xj[2 * a + 1];
                    im += (int64_t)xi[2 * a] * xj[2 * a + 1] - (int64_t)xi[2 * a + 1] * xj[2 * a];
                }
                int64_t *o = V + 2 * ((int64_t)k * B + (int64_t)i * (i + 1) / 2 + j);
                o[0] = re;
                o[1] = im;
            }
        }
        free(X);
    }
}

/* ------------------------------------------------------------------------- */
/* Requantisers                                                               */
/* ------------------------------------------------------------------------- */

/*
 * Round y to the nearest value of a binary floating-point format with
 * `mbits` stored mantissa bits and minimum normal exponent `emin`
 * (subnormals share the quantum 2^(emin - mbits)), ties to even, then
 * saturate magnitudes above `maxval` to `maxval`.  Returns the rounded value.
 *
 *   binary16  : mbits 10, emin -14, maxval 65504
 *   OCP E4M3  : mbits  3, emin  -6, maxval 448   (no infinities)
 *
 * The division by a power of two is exact and rint() rounds half to even in
 * the default rounding mode, so the only rounding is the one intended.
 */
double oracle_round_format(double y, int mbits, int emin, double maxval)
{
    if (y == 0.0 || isnan(y))
        return y;
    const double mag = fabs(y);
    int e2;
    frexp(mag, &e2);             /* mag = f * 2^e2, f in [0.5, 1) */
    int e = e2 - 1;              /* exponent of the leading bit */
    if (e < emin)
        e = emin;                /* subnormal range: fixed quantum */
    const double quantum = ldexp(1.0, e - mbits);
    double r = rint(mag / quantum) * quantum;
    if (r > maxval)
        r = maxval;
    return copysign(r, y);
}

void oracle_quant_f16(const double *y, int64_t n, double *q)
{
    for (int64_t t = 0; t < n; ++t)
        q[t] = oracle_round_format(y[t], 10, -14, 65504.0);
}

void oracle_quant_e4m3(const double *y, int64_t n, double *q)
{
    for (int64_t t = 0; t < n; ++t)
        q[t] = oracle_round_format(y[t], 3, -6, 448.0);
}

/* int8: q = clamp(rne(y), -127, 127); the symmetric range makes negation and
 * conjugation exact. */
void oracle_quant_int8(const double *y, int64_t n, int8_t *q)
{
    for (int64_t t = 0; t < n; ++t) {
        double r = rint(y[t]);
        if (r > 127.0)
            r = 127.0;
        if (r < -127.0)
            r = -127.0;
        q[t] = (int8_t)r;
    }
}

/*
 * Decoders from the format definitions, used to read reduced-precision
 * spectra back as numbers.
 *
 * OCP E4M3: sign bit 7, exponent bits 6..3 (bias 7), mantissa bits 2..0.
 * Exponent field 0 is subnormal (m/8 * 2^-6).  The pattern S.1111.111 is NaN;
 * there are no infinities, so S.1111.110 = 448 is the largest finite value.
 */
double oracle_decode_e4m3(int code)
{
    const int s = (code >> 7) & 1, E = (code >> 3) & 15, m = code & 7;
    double v;
    if (E == 15 && m == 7)
        v = NAN;
    else if (E == 0)
        v = ldexp((double)m / 8.0, -6);
    else
        v = ldexp(1.0 + (double)m / 8.0, E - 7);
    return s ? -v : v;
}

/* IEEE binary16: sign bit 15, exponent bits 14..10 (bias 15), mantissa 9..0. */
double oracle_decode_f16(int code)
{
    const int s = (code >> 15) & 1, E = (code >> 10) & 31, m = code & 1023;
    double v;
    if (E == 31)
        v = m ? NAN : INFINITY;
    else if (E == 0)
        v = ldexp((double)m / 1024.0, -14);
    else
        v = ldexp(1.0 + (double)m / 1024.0, E - 15);
    return s ? -v : v;
}
