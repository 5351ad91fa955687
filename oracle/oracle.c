/*
 * oracle.c -- plain FP64 CPU oracle of the F-engine channelizer.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the HIP product path never does
 * and shares no code with it.
 *
 * Every function follows one step of Sec. 2.1 of Merry, "Efficient
 * channelization on a Graphics Processing Unit", in the paper's order and
 * notation, written for clarity: scalar loops, double precision throughout,
 * a textbook radix-2 FFT whose twiddles come straight from libm.
 *
 * Readings of the paper where it is silent:
 *   - bit order of the packed 10-bit samples: MSB first within the sample,
 *     bytes filled MSB first (two's complement);
 *   - delay split: c = floor(d) + [frac(d) >= 0.5], tau = d - c (ties up);
 *     a delay whose c falls outside [0, max_delay] zeroes the spectrum;
 *   - spectrum labelling in Eq. (1): spectrum F has t0 = 2n(F - T + 1), so
 *     its window ends at 2n(F+1) - c and a call of N samples emits N/(2n)
 *     spectra; samples before the first sample of the stream are zero;
 *   - FFT: forward (negative exponent) and unnormalised;
 *   - fine delay: Y[k] = G[k] exp(i(phi - pi k tau / n)) X[k], i.e. a delay
 *     of tau samples at channel frequency k/(2n) cycles/sample, so coarse
 *     and fine delay together delay the signal by d;
 *   - quantisation: round half to even, saturate symmetrically to +-127,
 *     decided on the double-precision value itself.
 * Parity of these conventions is fixed by this reading, not by the paper.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ---- Step 1 (Sec. 2.1 item 1, Sec. 2.2): 10-bit signed samples ---------- */

int32_t oracle_sample10(const uint8_t *raw, int64_t i)
{
    int32_t code = 0;
    for (int b = 0; b < 10; ++b) {
        int64_t bit = 10 * i + b;                       /* position in the bitstream */
        int v = (raw[bit / 8] >> (7 - (int)(bit % 8))) & 1;
        code = 2 * code + v;                            /* MSB first */
    }
    return code >= 512 ? code - 1024 : code;            /* two's complement */
}

void oracle_unpack10(const uint8_t *raw, int64_t first, int64_t count, int32_t *out)
{
    for (int64_t i = 0; i < count; ++i)
        out[i] = oracle_sample10(raw, first + i);
}

/* ---- Steps 2 and 4 (Sec. 2.1 items 2 and 4, Sec. 3.3): delay split ------- */

int oracle_split_delay(double d, int64_t max_delay, int64_t *coarse, double *fine)
{
    double whole, frac, c;

    *coarse = 0;
    *fine = 0.0;
    if (!isfinite(d))
        return 0;
    whole = floor(d);
    frac = d - whole;
    c = (frac >= 0.5) ? whole + 1.0 : whole;
    if (c < 0.0 || c > (double)max_delay)
        return 0;
    *coarse = (int64_t)c;
    *fine = d - c;
    return 1;
}

/* ---- Step 3, Eq. (1): PFB FIR ------------------------------------------- */

int oracle_pfb_fir(const double *s, int64_t s_first, int64_t s_count, int n,
                   int taps, const float *h, int64_t F, int64_t coarse,
                   double *g)
{
    const int64_t two_n = 2 * (int64_t)n;
    const int64_t t0 = two_n * (F - taps + 1);          /* spectrum start time */

    for (int64_t t = 0; t < two_n; ++t) {
        double acc = 0.0;
        for (int j = 0; j < taps; ++j) {
            int64_t i = t0 + t - coarse + two_n * j;    /* s_{t0 + t - c + 2nj} */
            double x;
            if (i < 0) {
                x = 0.0;                                /* before the stream began */
            } else {
                if (i < s_first || i >= s_first + s_count)
                    return -1;
                x = s[i - s_first];
            }
            acc += x * (double)h[t + two_n * j];        /* w_{t,j} = h[t + 2nj] */
        }
        g[t] = acc;
    }
    return 0;
}

/* ---- Step 3: Fourier transform ------------------------------------------- */

int oracle_fft(double *re, double *im, int N)
{
    if (N < 1 || (N & (N - 1)))
        return -1;
    /* bit-reversal permutation */
    for (int i = 1, j = 0; i < N; ++i) {
        int bit = N >> 1;
        for (; j & bit; bit >>= 1)
            j ^= bit;
        j ^= bit;
        if (i < j) {
            double tr = re[i], ti = im[i];
            re[i] = re[j]; im[i] = im[j];
            re[j] = tr; im[j] = ti;
        }
    }
    /* butterflies, twiddle exp(-2 pi i k / len) from libm */
    for (int len = 2; len <= N; len <<= 1) {
        int half = len / 2;
        for (int k = 0; k < half; ++k) {
            double ang = -2.0 * M_PI * (double)k / (double)len;
            double wr = cos(ang), wi = sin(ang);
            for (int b = 0; b < N; b += len) {
                int p = b + k, q = b + k + half;
                double vr = re[q] * wr - im[q] * wi;
                double vi = re[q] * wi + im[q] * wr;
                re[q] = re[p] - vr;
                im[q] = im[p] - vi;
                re[p] = re[p] + vr;
                im[p] = im[p] + vi;
            }
        }
    }
    return 0;
}

int oracle_rfft_keep(const double *g, int n, double *X)
{
    int N = 2 * n, rc;
    double *re = malloc(sizeof(double) * (size_t)N);
    double *im = calloc((size_t)N, sizeof(double));
    if (!re || !im) {
        free(re);
        free(im);
        return -1;
    }
    memcpy(re, g, sizeof(double) * (size_t)N);
    rc = oracle_fft(re, im, N);
    for (int k = 0; k < n; ++k) {                       /* non-negative bins, no Nyquist */
        X[2 * k] = re[k];
        X[2 * k + 1] = im[k];
    }
    free(re);
    free(im);
    return rc;
}

/* ---- Steps 4 and 5 (Sec. 2.1 items 4 and 5, Sec. 3.6) -------------------- */

void oracle_fine_delay_gain(const double *X, int n, double tau, double phi,
                            const float *gain, double *Y)
{
    for (int k = 0; k < n; ++k) {
        double ang = phi - M_PI * (double)k * tau / (double)n;
        double cr = cos(ang), ci = sin(ang);
        double xr = X[2 * k], xi = X[2 * k + 1];
        double rr = cr * xr - ci * xi;                  /* phase rotation */
        double ri = cr * xi + ci * xr;
        double gr = gain[2 * k], gi = gain[2 * k + 1];  /* bandpass correction */
        Y[2 * k] = gr * rr - gi * ri;
        Y[2 * k + 1] = gr * ri + gi * rr;
    }
}

/* ---- Step 6 (Sec. 2.1 item 6, Sec. 3.6): quantisation and corner turn ---- */

int8_t oracle_quantize(double v)
{
    double r, diff;

    if (isnan(v))
        return 0;
    r = floor(v);
    diff = v - r;                                       /* exact in double */
    if (diff > 0.5 || (diff == 0.5 && fmod(r, 2.0) != 0.0))
        r += 1.0;                                       /* nearest, ties to even */
    if (r > 127.0)
        r = 127.0;                                      /* saturate */
    if (r < -127.0)
        r = -127.0;
    return (int8_t)r;
}

int oracle_heap_layout(const int8_t *q, int A, int64_t M, int n, int S,
                       int8_t *heap)
{
    if (S <= 0 || M % S)
        return -1;
    for (int a = 0; a < A; ++a)
        for (int p = 0; p < 2; ++p)
            for (int64_t F = 0; F < M; ++F)
                for (int k = 0; k < n; ++k)
                    for (int c = 0; c < 2; ++c) {
                        int64_t src = ((((int64_t)a * 2 + p) * M + F) * n + k) * 2 + c;
                        int64_t dst = (((((int64_t)a * (M / S) + F / S) * n + k) * S
                                        + F % S) * 2 + p) * 2 + c;
                        heap[dst] = q[src];
                    }
    return 0;
}

/* ---- The whole path ------------------------------------------------------- */

int64_t oracle_channelize(const uint8_t *raw, int64_t total, int A, int n,
                          int taps, int64_t max_delay, const float *weights,
                          const double *delays, const double *phases,
                          const float *gains, int64_t f_begin, int64_t f_end,
                          double *g_out, double *x_out, double *y_out,
                          int8_t *q_out, int8_t *valid_out)
{
    const int64_t two_n = 2 * (int64_t)n;
    const int64_t M = total / two_n;
    const int64_t nF = f_end - f_begin;
    const int64_t bytes = total * 10 / 8;
    int64_t invalid = 0;

    if (A < 1 || n < 1 || taps < 1 || max_delay < 0 || total % 4 || total % two_n
        || f_begin < 0 || f_end > M || f_begin > f_end)
        return -1;

    /* samples this range of spectra can read (window starts shifted by <= max_delay) */
    int64_t s_first = two_n * (f_begin - taps + 1) - max_delay;
    if (s_first < 0)
        s_first = 0;
    int64_t s_count = two_n * f_end - s_first;
    if (s_count < 0)
        s_count = 0;

    double *s = malloc(sizeof(double) * (size_t)(s_count > 0 ? s_count : 1));
    int32_t *si = malloc(sizeof(int32_t) * (size_t)(s_count > 0 ? s_count : 1));
    double *g = malloc(sizeof(double) * (size_t)two_n);
    double *X = malloc(sizeof(double) * (size_t)two_n);
    double *Y = malloc(sizeof(double) * (size_t)two_n);
    if (!s || !si || !g || !X || !Y) {
        invalid = -1;
        goto out;
    }

    for (int a = 0; a < A; ++a) {
        for (int p = 0; p < 2; ++p) {
            const int64_t sp = (int64_t)a * 2 + p;
            const uint8_t *stream = raw + sp * bytes;
            oracle_unpack10(stream, s_first, s_count, si);
            for (int64_t i = 0; i < s_count; ++i)
                s[i] = (double)si[i];

            for (int64_t f = 0; f < nF; ++f) {
                const int64_t F = f_begin + f;
                const int64_t o = sp * nF + f;          /* output spectrum index */
                int64_t c;
                double tau;
                int ok = oracle_split_delay(delays[sp * M + F], max_delay, &c, &tau);

                if (ok) {
                    if (oracle_pfb_fir(s, s_first, s_count, n, taps, weights, F, c, g)
                        || oracle_rfft_keep(g, n, X)) {
                        invalid = -1;
                        goto out;
                    }
                    oracle_fine_delay_gain(X, n, tau, phases[sp * M + F],
                                           gains + sp * 2 * n, Y);
                } else {
                    ++invalid;
                    memset(g, 0, sizeof(double) * (size_t)two_n);
                    memset(X, 0, sizeof(double) * (size_t)two_n);
                    memset(Y, 0, sizeof(double) * (size_t)two_n);
                }
                if (valid_out)
                    valid_out[o] = (int8_t)ok;
                if (g_out)
                    memcpy(g_out + o * two_n, g, sizeof(double) * (size_t)two_n);
                if (x_out)
                    memcpy(x_out + o * two_n, X, sizeof(double) * (size_t)two_n);
                if (y_out)
                    memcpy(y_out + o * two_n, Y, sizeof(double) * (size_t)two_n);
                if (q_out)
                    for (int64_t k = 0; k < two_n; ++k)
                        q_out[o * two_n + k] = oracle_quantize(Y[k]);
            }
        }
    }
out:
    free(s);
    free(si);
    free(g);
    free(X);
    free(Y);
    return invalid;
}
