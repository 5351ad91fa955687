/*
 * fengine.h -- C ABI of the MI355X (gfx950) F-engine channelizer.
 *
 * The library implements the wide-band channelizer data path of Sec. 2.1 of
 * Merry, "Efficient channelization on a Graphics Processing Unit": for each
 * polarization of each antenna it unpacks signed 10-bit samples (item 1),
 * applies the integer coarse delay by choosing where each PFB window is read
 * (item 2, Sec. 3.3), runs the polyphase filter bank -- the FIR of Eq. (1)
 * followed by a 2n-point real-to-complex FFT keeping channels 0..n-1 (item 3)
 * -- rotates each channel by the fine delay and phase (item 4), multiplies by
 * a complex per-channel gain (item 5), and quantizes to 8-bit signed
 * Gaussian integers with rounding and saturation, written channel-major
 * within each output heap of S_h spectra (item 6, Secs. 2.2 and 3.6).
 *
 * Conventions (the paper leaves these open; the library fixes them):
 *  - input: per polarization, a bitstream of 10-bit two's complement
 *    codes, MSB first, bytes filled MSB first (4 samples = 5 bytes);
 *  - delays: the total delay d_F (samples) of spectrum F splits into
 *    c = floor(d) + [d - floor(d) >= 0.5] and tau = d - c in [-0.5, 0.5);
 *    spectrum F's window is samples [2n(F-T+1) - c, 2n(F+1) - c) of the
 *    stream (so a call of N samples emits exactly N/(2n) spectra and the
 *    first T-1 spectra of a stream read zeros before its first sample);
 *  - w_{t,j} = h[t + 2nj] for the prototype filter h[0 .. 2nT);
 *  - Y[k] = G[k] * exp(i(phi_F - pi k tau_F / n)) * X[k], X the forward,
 *    unnormalised FFT;
 *  - q = clamp(round_half_even(Re/Im Y), -127, 127);
 *  - output of one call: int8 [A][M/S_h][n][S_h][2 pols][re, im].
 *
 * All functions return fe_status (0 on success, < 0 on error); no C++
 * exception crosses the ABI.  Device pointers are HIP device allocations on
 * the device that was current when the stream was created; the caller owns
 * every buffer passed in and must keep it alive until the work enqueued on
 * the stream's HIP stream has finished.
 */
#ifndef FENGINE_H
#define FENGINE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fe_status;

enum {
    FE_OK = 0,
    FE_EINVAL = -1,   /* bad argument: null pointer, size not a multiple of
                         2n*S_h, unsupported n or T, ... (nothing enqueued) */
    FE_ENOMEM = -2,   /* device allocation failed (fe_stream_create only) */
    FE_EHIP = -3,     /* a HIP runtime call or kernel launch failed */
    FE_EDELAY = -4,   /* sticky device-side status: some spectrum's coarse
                         delay fell outside [0, max_delay] or its delay was
                         not finite; that polarization's spectrum was written
                         as zeros.  Reported by fe_stream_status. */
    FE_ESIZE = -5     /* n_samples larger than the stream's max_samples */
};

/* Arithmetic of the FIR and FFT (fe_config.precision).
 *   FE_PREC_FP32  float32 throughout (the reference path).
 *   FE_PREC_FP16  the FIR of Eq. (1) and the radix-16 DFT stages run on the
 *                 matrix cores with FP16 operands and FP32 accumulation; the
 *                 filtered samples pass between kernels as FP16.  The
 *                 10-bit samples are exact in FP16; the taps are scaled by a
 *                 power of two so that none falls into the FP16 subnormal
 *                 range.  Pre-quantisation error ~4e-4 relative (normwise).
 *                 Above 8192 channels the filter runs on the vector ALUs and
 *                 hands the two-level FFT, which runs in float32, its input
 *                 as FP16 pairs (FP16 storage, float32 arithmetic; Sec. 6 of
 *                 the paper suggests exactly that split).
 *   FE_PREC_BF16  the same contractions with BF16 operands, each split into
 *                 a high and a low BF16 part (three products per term); the
 *                 filtered samples pass as FP32.
 * Twiddles, phases and the delay split are computed in FP64 in every mode.
 * Sec. 3.5.1 of the paper keeps its FFT in FP32 because an FP16 FFT leaves
 * data-dependent spurs near -75 dB; the reduced modes trade that for speed
 * and are measured against the FP64 oracle stage by stage. */
enum { FE_PREC_FP32 = 0, FE_PREC_FP16 = 1, FE_PREC_BF16 = 2 };

/* Stream configuration, fixed at creation.
 *   n_channels        n: a power of two, 256 .. 32768 (FE_PREC_FP32, FE_PREC_FP16),
 *                     256 .. 8192 (FE_PREC_BF16); above 8192 the FFT runs in two
 *                     levels (a radix-16 pass, then n/16-point transforms)
 *   taps              T: 1 .. 32
 *   n_antennas        A >= 1; every antenna has two polarizations
 *   spectra_per_heap  S_h >= 1 (256 in the paper, Sec. 2.2)
 *   max_delay         D_max >= 0, largest coarse delay accepted (samples)
 *   precision         one of FE_PREC_* (0 = FP32)
 *   max_samples       largest N (samples per polarization) of one call,
 *                     a multiple of 2n*S_h, at most 2^28; sizes the
 *                     library's workspace (A*2*max_samples*5 bytes)
 *   weights           HOST pointer to float32[2n*T], the prototype filter h;
 *                     copied to the device during fe_stream_create */
typedef struct fe_config {
    int32_t n_channels;
    int32_t taps;
    int32_t n_antennas;
    int32_t spectra_per_heap;
    int32_t max_delay;
    int32_t precision;
    int64_t max_samples;
    const float *weights;
} fe_config;

/* Opaque per-stream state owned by the library: the last
 * 2n(T-1)+D_max samples of every polarization (the overlap of Sec. 3.1,
 * enlarged for delay changes as in Sec. 3.3), the device copy of the
 * weights, the workspace and the sticky status word. */
typedef struct fe_stream fe_stream;

/* Create a stream whose work is enqueued on `hip_stream` (a hipStream_t,
 * NULL for the default stream).  The history starts as zeros (samples before
 * the stream's first sample read as zero).  Allocates device memory and
 * synchronizes once; *out is set only on success. */
fe_status fe_stream_create(const fe_config *cfg, void *hip_stream, fe_stream **out);

/* Release a stream (synchronizes its HIP stream first).  NULL is accepted. */
fe_status fe_stream_destroy(fe_stream *s);

/* Change the HIP stream later calls are enqueued on. */
fe_status fe_stream_set_hip_stream(fe_stream *s, void *hip_stream);

/* Enqueue: zero the history, clear the sticky status, restart at sample 0. */
fe_status fe_stream_reset(fe_stream *s);

/* Channelize the next N samples of every polarization (Sec. 2.1, items 1-6).
 *   raw     device uint8 [A][2][N*5/4]: the packed samples of this call,
 *           continuing where the previous call of this stream stopped
 *   n_samples  N > 0, a multiple of 2n*S_h, <= max_samples
 *   delays  device float64 [A][2][M], M = N/(2n): total delay d_F (samples)
 *           of each spectrum of this call
 *   phases  device float64 [A][2][M]: phase phi_F (radians)
 *   gains   device float32 [A][2][n][2]: complex gain (re, im) per channel
 *   out     device int8 [A][M/S_h][n][S_h][2][2]
 * Enqueues the work and returns without synchronizing and without
 * allocating.  Not safe to call on one fe_stream from two host threads at
 * once.  On FE_EINVAL/FE_ESIZE nothing is enqueued and the stream state is
 * unchanged. */
fe_status fe_channelize(fe_stream *s, const uint8_t *raw, int64_t n_samples,
                        const double *delays, const double *phases,
                        const float *gains, int8_t *out);

/* The same call with the pre-quantisation spectra as output:
 *   y_out   device float32 [A][2][M][n][2] = Y (complex64)
 * Identical kernels, identical state update; only the final store differs. */
fe_status fe_channelize_prequant(fe_stream *s, const uint8_t *raw, int64_t n_samples,
                                 const double *delays, const double *phases,
                                 const float *gains, float *y_out);

/* The same call stopped after the FIR (Eq. (1)):
 *   g_out   device float32 [A][2][M][2n], the filtered samples g of every
 *           spectrum (zeros where the delay was out of range); for an
 *           FE_PREC_FP16 stream the values are rounded to FP16, which up to
 *           8192 channels is what the FFT reads (above, the FFT reads the
 *           first radix-16 stage's output rounded to FP16).
 * Updates the stream state exactly as fe_channelize does. */
fe_status fe_channelize_fir(fe_stream *s, const uint8_t *raw, int64_t n_samples,
                            const double *delays, float *g_out);

/* Bytes of the static device scratch of fe_channelize_noalloc, on every GPU
 * the library runs on. */
#define FE_NOALLOC_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * call, output and stream-state update as fe_channelize, with the call's
 * intermediate buffers (filtered samples, int8 spectra before the corner
 * turn, the two-level FFT's reordered gains, the history assembly of calls
 * shorter than the history) in a static device array of the library,
 * FE_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends, instead of
 * the stream's workspace.  Allocates nothing and does not synchronize.  A
 * call needs 4 bytes per real sample for the filtered samples (none on the
 * fused path), 1 byte per real sample for the int8 spectra, 16n bytes per
 * antenna when n > 8192 and 2.5 H bytes per antenna when n_samples < H,
 * each rounded up to 256 bytes; a call needing more than
 * FE_NOALLOC_SCRATCH_BYTES returns FE_ESIZE before anything is enqueued.
 * Every call on one GPU shares that GPU's scratch: calls that overlap on one
 * GPU (on different HIP streams, or from several host threads) race and
 * corrupt each other's results; calls enqueued on one HIP stream are
 * ordered and safe.  No part of the scratch is read before the call writes
 * it, so nothing needs clearing between calls. */
fe_status fe_channelize_noalloc(fe_stream *s, const uint8_t *raw, int64_t n_samples,
                                const double *delays, const double *phases, const float *gains,
                                int8_t *out);

/* Synchronize the stream's HIP stream and return its sticky status:
 * FE_OK, FE_EDELAY (cleared only by fe_stream_reset), or FE_EHIP. */
fe_status fe_stream_status(fe_stream *s);

/* Kernel timing for measurement tools.  While enabled, every call records
 * HIP events on its HIP stream around its kernels (no synchronization, no
 * device allocation; events are created by fe_stream_timing(s, 1), at most
 * 4096 calls are recorded between reads).  fe_stream_timing_read
 * synchronizes and returns, over the calls recorded since timing was enabled
 * or last read, the summed milliseconds of the FIR kernel (steps 1-3a), of
 * the FFT/post-processing kernel (steps 3b-6 up to the int8 values) and of the
 * corner turn into heaps, and the number of calls, then starts a new
 * accumulation.  Any pointer may be NULL. */
fe_status fe_stream_timing(fe_stream *s, int enable);
fe_status fe_stream_timing_read(fe_stream *s, double *fir_ms, double *post_ms, double *turn_ms,
                                int64_t *calls);

/* Test hook for step 1 alone: unpack samples [first, first+count) of the
 * packed stream `raw` (device, at least (first+count)*10/8 rounded up bytes)
 * into int32 `out` (device) with the library's device unpacker, on
 * `hip_stream`.  first and count >= 0. */
fe_status fe_debug_unpack10(const uint8_t *raw, int64_t first, int64_t count,
                            int32_t *out, void *hip_stream);

/* ---- Tuning ------------------------------------------------------------- */

/* Time the stream's launch choices on the caller's buffers (an fe_channelize
 * call's arguments; `iters` timed calls per candidate, HIP events on the
 * stream's HIP stream) and keep the fastest.  Each path the stream can run
 * (fe_stream_set_schedule: FP32 split, split with the turn folded, fused;
 * FP16/BF16 on the vector FIR split or folded) is timed, and the fastest
 * kept; their results are identical bit for bit.  The FIR engine of an
 * FP16/BF16 stream is not changed (it changes the rounding).  The
 * candidates set the FIR's schedule: for FP32 streams its run length -- how many consecutive batches
 * of spectra one workgroup filters (a batch is 64 spectra, 48 for 24 taps),
 * trading tap reloads against parallelism; for FP16/BF16 streams the chain
 * length of the matrix-core FIR -- how many consecutive 256-spectrum tiles
 * one workgroup walks (its taps loaded once, each tile's rows fetched during
 * the previous tile's contraction).  Candidates: 1, 2, 4, 8, or the
 * per-launch default.  Then, for streams above 8192 channels, the split of
 * the two-level FFT's post kernel (fe_stream_set_fft_parts: 1, 3 or 9
 * workgroups per spectrum, or the per-call default) is timed the same way.
 * The timing calls advance the stream like real calls, so the stream is
 * reset (fe_stream_reset) before returning.  Synchronizes.  *choice (may be
 * NULL) receives the chosen run length (0 = per-launch default). */
fe_status fe_stream_autotune(fe_stream *s, const uint8_t *raw, int64_t n_samples,
                             const double *delays, const double *phases, const float *gains,
                             int8_t *out, int iters, int *choice);

/* Set the FIR schedule directly (0 = per-launch default, else 1..64:
 * batches of spectra per run (FP32) or tiles per chain (FP16/BF16), as
 * above). */
fe_status fe_stream_set_tuning(fe_stream *s, int fir_batches);

/* Streams above 8192 channels: the two-level FFT's post kernel transforms a
 * spectrum's 16 sub-transforms in nine rounds (pairs d, 16 - d); `parts`
 * workgroups share them (1 .. 9; 0 = chosen per call: 9 for calls of under
 * 128 spectra-polarizations, 3 under 512, else 1).  Results are identical
 * bit for bit for every value; ignored at 8192 channels and below.
 * FE_EINVAL for parts outside 0 .. 9. */
fe_status fe_stream_set_fft_parts(fe_stream *s, int parts);
/* The current setting (0 = per call). */
fe_status fe_stream_get_fft_parts(const fe_stream *s, int *parts);

/* Kernels of the path (fe_stream_set_schedule). */
enum { FE_PATH_AUTO = 0, FE_PATH_SPLIT = 1, FE_PATH_FUSED = 2, FE_PATH_MATRIX_FIR = 3, FE_PATH_SPLIT_FOLDED = 4 };

/* Choose the kernels that run a stream's calls, and the FIR schedule.
 * FE_PATH_SPLIT: a FIR kernel (steps 1-3a) writes the filtered samples as
 *   float32 to the stream's workspace, an FFT/post-processing kernel
 *   (steps 3b-6) reads them back, a corner-turn kernel writes the heaps.
 * FE_PATH_FUSED (FP32 streams with n <= 4096 and T <= 16 only): one kernel
 *   filters four consecutive spectra of a polarization into on-chip memory
 *   and transforms and finishes them there; no filtered sample is written to
 *   device memory.  Then the corner turn.
 * FE_PATH_MATRIX_FIR (FP16/BF16 streams only): the split path with the FIR
 *   on the matrix cores as a banded Toeplitz contraction (16 consecutive
 *   spectra of a column per v_mfma_f32_16x16x32, taps in FP16 or BF16
 *   hi + lo).  Otherwise FP16/BF16 streams filter on the vector ALUs in
 *   float32 and store the filtered samples as FP16 (FP16 streams) or float32
 *   (BF16 streams) for the matrix-core DFT stages.
 * FE_PATH_SPLIT_FOLDED (streams with n <= 8192, FP16/BF16 ones on the
 *   vector FIR; others run the split path): the split path without the
 *   corner-turn kernel.  Each FFT/post workgroup (float32, or with the
 *   matrix-core DFT stages) transforms both polarizations of one or two consecutive
 *   spectra and writes every channel's bytes straight into the heap (Sec.
 *   3.6 turns inside its post-processing kernel too): 2 bytes per sample
 *   less device-memory traffic, one launch fewer.
 * FE_PATH_AUTO: fused for FP32 streams with T <= 8 and n <= 2048; split
 *   with the turn folded for other FP32 streams with n <= 8192 whose calls
 *   give the folded kernel at least 8 workgroups per compute unit (on MI355X
 *   as fast as the separate turn, with 2 bytes per sample less traffic);
 *   else split (FP16/BF16 streams: their folded kernel is as fast as the
 *   split pair, not faster; fe_stream_autotune times both).  The schedule
 *   reported for FE_PATH_AUTO is that of a call of max_samples.
 * Streams the fused path cannot run always run the split path (the setting
 * is kept).  fir_batches as in fe_stream_set_tuning; on the fused path it
 * caps the kernel's workgroups per compute unit (0 = as many as fit).
 * fe_stream_autotune chooses both.  FE_EINVAL for an unknown path or
 * fir_batches outside 0..64. */
fe_status fe_stream_set_schedule(fe_stream *s, int path, int fir_batches);

/* The path the stream's calls run now (FE_PATH_SPLIT, FE_PATH_FUSED,
 * FE_PATH_MATRIX_FIR or FE_PATH_SPLIT_FOLDED) and its fir_batches setting.  Either pointer may be
 * NULL. */
fe_status fe_stream_get_schedule(const fe_stream *s, int *path, int *fir_batches);

/* ---- Batches of streams ------------------------------------------------ */

/* One member's fe_channelize arguments. */
typedef struct fe_call {
    const uint8_t *raw;
    int64_t n_samples;
    const double *delays;
    const double *phases;
    const float *gains;
    int8_t *out;
} fe_call;

/* A batch runs one call of every member stream (streams of any n, T, A and
 * precision) as a unit: each member's kernels go to a fork HIP stream of its
 * own, forked from and joined back into the batch's HIP stream, so the
 * members' work overlaps on the device.  fe_batch_capture records that unit
 * for fixed buffers into a HIP graph; each fe_batch_launch then replays it
 * with a single graph launch (every member advancing by one call, state
 * included).  The members stay owned by the caller and must outlive the
 * batch; while a batch runs them, they must not be used directly. */
typedef struct fe_batch fe_batch;

/* members: `count` streams; hip_stream: the batch's HIP stream (NULL =
 * default stream).  Creates the fork streams (default priority). */
fe_status fe_batch_create(fe_stream *const *members, int count, void *hip_stream, fe_batch **out);

/* Synchronize and release (not the members).  NULL is accepted. */
fe_status fe_batch_destroy(fe_batch *b);

/* Enqueue one call per member now (calls[i] for member i; no graph). */
fe_status fe_batch_run(fe_batch *b, const fe_call *calls);

/* Record one call per member with these buffers into the batch's graph
 * (replacing an earlier one).  Synchronizes the batch stream first; nothing
 * runs until fe_batch_launch.  The buffers must stay valid while the graph
 * is used. */
fe_status fe_batch_capture(fe_batch *b, const fe_call *calls);

/* Replay the captured graph on the batch stream (FE_EINVAL if none). */
fe_status fe_batch_launch(fe_batch *b);

/* How a batch step is issued (default 0: every member's kernels on a fork
 * stream of its own, which measures faster on MI355X for uneven batches:
 * 243.6 against 227.7 Gsample/s on 16 streams of 1024-32768 channels).
 * Grouped (1): the FP32
 * members on the split path (fe_stream_set_schedule) run through kernels
 * driven by job lists spanning the members -- per step one seam-staging
 * copy, one FIR launch per (kernel) tap count, one history copy, one
 * FFT/post launch per channel count up to 8192 (larger channel counts run
 * their two-level FFT per member), one corner-turn launch -- on the batch's
 * HIP stream, while every other member (fused path, FP16/BF16) runs on a
 * fork stream of its own.  The job lists live in device tables the batch
 * owns: fe_batch_capture writes the graph's table before capturing,
 * fe_batch_run uploads its own from pinned host memory on the batch stream
 * (waiting first for the previous run's upload).  Outputs are the same
 * either way. */
fe_status fe_batch_set_grouped(fe_batch *b, int grouped);

/* Human-readable text of a status code (static storage). */
const char *fe_strerror(fe_status status);

/* Library version, major*10000 + minor*100 + patch. */
int32_t fe_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FENGINE_H */
