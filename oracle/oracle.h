/*
 * oracle.h -- plain FP64 CPU oracle of the F-engine channelizer.
 *
 * TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg are the only users.  The HIP implementation
 * never includes, links or loads it, and shares no code with it.
 *
 * Notation (Sec. 2.1 of Merry, "Efficient channelization on a Graphics
 * Processing Unit"): n channels, a 2n-point real FFT, T taps, prototype
 * filter h[0 .. 2nT) with PFB weights w_{t,j} = h[t + 2nj], coarse delay c,
 * fine delay tau, phase phi, complex gain G.  Complex arrays are interleaved
 * (re, im) doubles or floats.
 */
#ifndef FENGINE_ORACLE_H
#define FENGINE_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Step 1: sample i of a packed, MSB-first, two's complement 10-bit stream. */
int32_t oracle_sample10(const uint8_t *raw, int64_t i);
void oracle_unpack10(const uint8_t *raw, int64_t first, int64_t count, int32_t *out);

/* Steps 2 and 4: split a total delay d into the coarse integer c and the
 * fine residual tau = d - c in [-0.5, 0.5).  Returns 1 if 0 <= c <= max_delay
 * (and d is finite), else 0 with c = 0, tau = 0. */
int oracle_split_delay(double d, int64_t max_delay, int64_t *coarse, double *fine);

/* Step 3, Eq. (1): the 2n filtered samples g[0..2n) of spectrum F of one
 * stream whose samples are s[i - s_first] for absolute index i >= s_first
 * (s holds s_count values); absolute indices below 0 read as zero.  The
 * window of spectrum F starts at absolute sample 2n(F - T + 1) - coarse.
 * Returns 0, or -1 if the window reaches outside [min(0,s_first), s_first+s_count). */
int oracle_pfb_fir(const double *s, int64_t s_first, int64_t s_count, int n,
                   int taps, const float *h, int64_t F, int64_t coarse,
                   double *g);

/* Forward, unnormalised DFT X[k] = sum_t x[t] exp(-2 pi i t k / N), in place,
 * N a power of two (textbook radix-2).  Returns 0, -1 if N is not a power of 2. */
int oracle_fft(double *re, double *im, int N);

/* Step 3: 2n-point real-to-complex transform of g, keeping k = 0 .. n-1
 * (the Nyquist bin is dropped).  X is n interleaved complex values. */
int oracle_rfft_keep(const double *g, int n, double *X);

/* Steps 4 and 5: Y[k] = G[k] * exp(i*(phi - pi*k*tau/n)) * X[k]. */
void oracle_fine_delay_gain(const double *X, int n, double tau, double phi,
                            const float *gain, double *Y);

/* Step 6: signed 8-bit value of v: the nearest integer to v (ties to even),
 * saturated to [-127, 127]. */
int8_t oracle_quantize(double v);

/* Step 6 corner turn: q[a][p][F][k][2] -> heap[a][F/S][k][F%S][p][2]. */
int oracle_heap_layout(const int8_t *q, int A, int64_t M, int n, int S,
                       int8_t *heap);

/* The whole path for spectra [f_begin, f_end) of A dual-pol antennas.
 *   raw    [A][2][total*5/4]  packed streams from their first sample
 *   delays [A][2][total/2n]   d_F per stream spectrum (global index F)
 *   phases [A][2][total/2n]   phi_F, radians
 *   gains  [A][2][n][2]       complex gain
 * Optional outputs (NULL to skip), nF = f_end - f_begin:
 *   g_out [A][2][nF][2n], x_out/y_out [A][2][nF][n][2], q_out [A][2][nF][n][2],
 *   valid_out [A][2][nF] (1, or 0 when the delay was out of range: that
 *   spectrum's outputs are zero).
 * Returns the number of invalid spectra, or -1 on bad arguments. */
int64_t oracle_channelize(const uint8_t *raw, int64_t total, int A, int n,
                          int taps, int64_t max_delay, const float *weights,
                          const double *delays, const double *phases,
                          const float *gains, int64_t f_begin, int64_t f_end,
                          double *g_out, double *x_out, double *y_out,
                          int8_t *q_out, int8_t *valid_out);

#ifdef __cplusplus
}
#endif

#endif
