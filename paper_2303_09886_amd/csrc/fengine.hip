// fengine.hip -- MI355X (gfx950) F-engine channelizer: kernels and C ABI.
//
// Data path (Sec. 2.1 of Merry, "Efficient channelization on a Graphics
// Processing Unit"), per polarization of each antenna:
//   1. unpack signed 10-bit samples                       (item 1, Sec. 2.2)
//   2. coarse delay = choice of where each window is read (item 2, Sec. 3.3)
//   3. PFB: FIR of Eq. (1), 2n-point real FFT, keep n bins (item 3)
//   4. fine delay as a per-channel phase rotation         (item 4, Sec. 3.6)
//   5. complex per-channel gain                           (item 5)
//   6. int8 quantisation, channel-major heaps             (item 6, Sec. 3.6)
//
// Two kernels per call:
//   fir_kernel      steps 1-3a.  One thread per FIR column t (Sec. 3.4: the
//                   input viewed as a 2n-wide matrix, column t filtered with
//                   weights w_t), sliding over a run of consecutive spectra
//                   with the window held in registers, so every packed
//                   sample is unpacked about once.  Writes float32 g.
//   fft_post_kernel steps 3b-6.  One workgroup per (antenna, spectrum): both
//                   polarizations' n-point complex FFTs (even/odd samples as
//                   re/im, the real-input technique of Sec. 4.1) in LDS with
//                   radix-16 Stockham passes, the real-FFT untangle, phase,
//                   gain, half-even rounding with saturation and the
//                   channel-major store.
// plus a small history copy: the last H = 2n(T-1)+D_max samples of every
// polarization stay on the device for the next call (the chunk overlap of
// Sec. 3.1 sized for delay changes as in Sec. 3.3).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "fengine.h"

namespace {

// ---------------------------------------------------------------------------
// Small complex helpers (float2 = re, im)
// ---------------------------------------------------------------------------

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
// multiply by -i
__device__ __forceinline__ float2 cmul_mi(float2 a) { return make_float2(a.y, -a.x); }

// Non-temporal (streaming, read-once) load of a complex value.
__device__ __forceinline__ float2 load_nt(const float2 *p)
{
    typedef float v2f __attribute__((ext_vector_type(2)));
    const v2f v = __builtin_nontemporal_load(reinterpret_cast<const v2f *>(p));
    return make_float2(v.x, v.y);
}

// ---------------------------------------------------------------------------
// Step 1: sample j (>= 0) of a packed, MSB-first 10-bit two's complement
// stream.  The 10 bits of a sample lie in bytes 5j/4 and 5j/4 + 1, starting
// at bit offset (10j) mod 8 = 2 (j mod 4) from the MSB.  Valid for
// j < 2^32 / 5.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int sample10(const uint8_t *__restrict__ p, uint32_t j)
{
    const uint32_t byte = (5u * j) >> 2;
    const uint32_t sh = (j & 3u) << 1;
    const uint32_t v = (uint32_t(p[byte]) << 8) | uint32_t(p[byte + 1]);
    return int32_t(v << (16u + sh)) >> 22;          // sign-extend the 10-bit field
}

// Sample at index i relative to the first sample of this call: i < 0 reads
// the history buffer, which holds the H samples preceding the call.
__device__ __forceinline__ int sample_at(const uint8_t *__restrict__ chunk,
                                         const uint8_t *__restrict__ hist,
                                         int64_t i, int H)
{
    return i >= 0 ? sample10(chunk, uint32_t(i)) : sample10(hist, uint32_t(i + H));
}

// ---------------------------------------------------------------------------
// Steps 2 and 4: split of the total delay d (float64) into the coarse integer
// c and the fine residual tau = d - c in [-0.5, 0.5):
//   c = floor(d) + [d - floor(d) >= 0.5]; valid iff d finite and 0 <= c <= D.
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool split_delay(double d, int D, int &c, double &tau)
{
    c = 0;
    tau = 0.0;
    // -0.5 <= d < D + 0.5 is exactly 0 <= c <= D and rejects NaN and inf
    if (!(d >= -0.5 && d < double(D) + 0.5))
        return false;
    const double whole = floor(d);
    const double frac = d - whole;
    const double cc = frac >= 0.5 ? whole + 1.0 : whole;
    c = int(cc);
    tau = d - cc;
    return true;
}

// Wavefront dispatch sends workgroup b to XCD b mod 8.  Map it to a logical
// index so that each XCD works on one contiguous range of logical indices:
// neighbouring tiles then share an L2 (which merges their partial writes to
// the same lines and serves the input bytes they share).
__device__ __forceinline__ int xcd_logical(int b, int G)
{
    constexpr int X = 8;
    const int xcd = b % X, local = b / X;
    const int per = (G + X - 1) / X;
    int full = G % X;
    if (full == 0)
        full = X;
    return xcd < full ? xcd * per + local : full * per + (xcd - full) * (per - 1) + local;
}

// ---------------------------------------------------------------------------
// Kernel 1: unpack + coarse delay + FIR (Eq. (1)).
//
// Thread = two adjacent columns t, t+1 (t even) of one stream (antenna, pol)
// for a run of R consecutive spectra.
//   g_{F,t} = sum_j s[2n(F-T+1) - c_F + t + 2nj] h[t+2nj].
// Viewed down a column, spectrum F reads rows F-T+1 .. F of the 2n-wide
// sample matrix shifted by c_F, so consecutive spectra with equal c share
// T-1 rows and each new spectrum needs one new row.  A row's two samples of
// the pair, i = 2n r - c + t and i + 1 (20 bits), lie in the 4 bytes from
// byte floor(5 i / 4): one unaligned dword load brings both, a byte swap and
// two sign-extending bitfield extracts unpack them, and the two outputs
// leave in one 8-byte (FP16: 4-byte) store.  (With one column per thread the
// kernel issues twice the vector memory instructions, and their address
// processing, not HBM, bounds it.)  Spectra go in groups of G = T (T < 8), 8
// (T <= 16) or 4: a group's G new rows are loaded together (memory-level
// parallelism), one group ahead of their use, and its G outputs per column
// come from a (T-1+G)-row register window.  The workgroup first splits the
// delays of up to FIR_SEG spectra into an LDS table (one per thread).  Each
// wave then walks the spectra in spans of one delay (found with one table
// read per lane and a ballot): a span's groups start at its first spectrum
// and its last group is padded (the padding outputs are not stored), so a
// delay step costs one refill of the T-1 older rows and part of one group.
// Spectra with an invalid delay or rows before the region take a general
// per-spectrum path.  The region's last row is read from one byte earlier by
// the one lane whose pair ends the region (its dword would pass the end by
// a byte), and the word is shifted back.
// ---------------------------------------------------------------------------

constexpr int FIR_THREADS = 256;
constexpr int FIR_SEG = 1024;              // spectra per delay table

// Raw buffer descriptor (gfx9 family): base, no stride, `bytes` records;
// loads outside [0, bytes) return zero, stores outside are dropped.  Used for
// aligned stores only (buffer loads at unaligned byte addresses do not
// behave like unaligned global loads).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, int(bytes), 0x00020000);
}

// How the FIR stores its filtered samples g: float32 (FP32 and BF16 streams),
// FP16 (FP16 streams: the matrix-core FFT's operand), or float32 holding the
// FP16-rounded value (FP16 streams' FIR-stage debug output).
enum { G_F32 = 0, G_F16 = 1, G_F32_AS_F16 = 2 };

// Unaligned 32-bit global load (little-endian) at byte `off` of a
// wave-uniform base in the global address space (so the address is an SGPR
// pair plus one 32-bit VGPR).
typedef const uint8_t __attribute__((address_space(1))) *gptr8;
typedef uint32_t __attribute__((aligned(1))) u32_unaligned;
__device__ __forceinline__ uint32_t load_u32u(gptr8 base, uint32_t off)
{
    return *reinterpret_cast<const u32_unaligned __attribute__((address_space(1))) *>(base + off);
}

// Store two filtered samples (columns t, t+1) through a buffer descriptor,
// non-temporally (cache policy 2: they stream to memory without displacing
// the taps and input rows from L2); the builtins' payloads are integers, so
// the bits are passed, not converted values.
typedef unsigned int v2u32 __attribute__((ext_vector_type(2)));

// workgroups per CU the register budget allows (two columns' windows)
#define FIR_WG_PER_CU(T) ((T) <= 8 ? 4 : (T) <= 16 ? 3 : 2)

// One complex value as an FP16 pair (round to nearest even) and back.
__device__ __forceinline__ uint32_t f16_pair(float2 v)
{
    return uint32_t(__builtin_bit_cast(uint16_t, (_Float16)v.x))
           | (uint32_t(__builtin_bit_cast(uint16_t, (_Float16)v.y)) << 16);
}
__device__ __forceinline__ float2 f16_unpair(uint32_t w)
{
    return make_float2(float(__builtin_bit_cast(_Float16, uint16_t(w))),
                       float(__builtin_bit_cast(_Float16, uint16_t(w >> 16))));
}

template <int GM>
__device__ __forceinline__ void store_g2(float a, float b, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    if constexpr (GM == G_F16) {
        const uint32_t w = uint32_t(__builtin_bit_cast(uint16_t, (_Float16)a))
                           | (uint32_t(__builtin_bit_cast(uint16_t, (_Float16)b)) << 16);
        __builtin_amdgcn_raw_buffer_store_b32(w, r, voff, soff, 2);
    } else {
        if constexpr (GM == G_F32_AS_F16) {
            a = float((_Float16)a);
            b = float((_Float16)b);
        }
        const v2u32 v = {__builtin_bit_cast(uint32_t, a), __builtin_bit_cast(uint32_t, b)};
        __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, 2);
    }
}

// spectra per group of the FIR: T (T < 8), 8 (T <= 16), 4
__host__ __device__ constexpr int fir_group(int T) { return T < 8 ? T : (T <= 16 ? 8 : 4); }

template <int R> struct Dft;               // small DFTs (defined with the FFT below)

// FRONT (FP32, n > 8192): the first radix-16 stage of the two-level FFT
// folded into the FIR.  Thread (j, gl) of the workgroup filters column pair
// gam + (n/16) j of the block's 16 groups gam = 16 cb + gl; a group's G rows
// of filtered samples go to the LDS tile `fl` [G][16 j][16 gl (+1 pad)], and
// after a barrier 16 G threads each take one (row, gam), form the DFT-16 over
// j, multiply output d by exp(-2 pi i gam d / n) (table `twf`, [n/16][16]) and
// store it at gam + (n/16) d: the rows fft_front_kernel would produce,
// without its read and write of g.
template <int T, int GM = G_F32, bool FRONT = false>
__device__ __forceinline__ void fir_block(
    int lb, int *__restrict__ s_c,
    const uint8_t *__restrict__ raw, int64_t raw_stride,
    const uint8_t *__restrict__ hist, int64_t hist_stride, int H,
    const float *__restrict__ taps, const double *__restrict__ delays,
    void *__restrict__ g, int n2, int M, int D, int R, int colblocks, int runs, int mb, int me,
    int moff, int mrows, float2 (*__restrict__ fl)[16][17] = nullptr, const float2 *__restrict__ twf = nullptr)
{
    constexpr int G = fir_group(T);                           // spectra per group
    constexpr uint32_t ES = GM == G_F16 ? 2u : 4u;          // bytes per stored sample
    static_assert(!FRONT || GM == G_F32 || GM == G_F16, "the folded front stage stores float32 or FP16 pairs");
    const int cb = lb % colblocks;
    const int rest = lb / colblocks;
    const int run = rest % runs;
    const int s = rest / runs;
    const int tid = threadIdx.x, lane = tid & 63;
    const int gpt = n2 / 32;                                  // FRONT: groups gam per spectrum (n/16)
    const int gbase = cb * 16;                                // FRONT: the block's first group
    // the block's smallest column, and the pair's first column
    const int t_blk = FRONT ? 2 * gbase : cb * 2 * FIR_THREADS;
    const int t = FRONT ? 2 * (gbase + (tid & 15) + gpt * (tid >> 4)) : t_blk + 2 * tid;
    const int m0 = mb + run * R;
    const int mend = min(m0 + R, me);

    float2 h[T];
#pragma unroll
    for (int j = 0; j < T; ++j)
        h[j] = *reinterpret_cast<const float2 *>(taps + t + n2 * j);

    const double *ds = delays + int64_t(s) * M;
    const uint8_t *rs = raw + int64_t(s) * raw_stride;
    const uint8_t *hs = hist + int64_t(s) * hist_stride;
    uint8_t *gs = static_cast<uint8_t *>(g) + int64_t(s) * M * n2 * ES;
    const __amdgpu_buffer_rsrc_t rg = make_rsrc(gs, uint32_t(int64_t(M) * n2 * ES));
    const int row_bytes = (n2 / 4) * 5;
    const uint32_t region_bytes = uint32_t(mrows) * uint32_t(row_bytes);
    const uint32_t t_bytes = uint32_t(t) * ES;

    // X0, X1: rows g0-T+1 .. g0-1 of the two columns at delay c_cur; W: the
    // raw words of rows g0 .. g0+G-1, loaded one group ahead of their use
    float X0[T - 1], X1[T - 1];
#pragma unroll
    for (int i = 0; i < T - 1; ++i)
        X0[i] = X1[i] = 0.f;
    int c_cur = -1;
    uint32_t W[G];
    // 1: this lane's word in the region's last row would end past the
    // region, so at this delay it reads every row's word a byte early (its
    // pair starts at bit 2 phi <= 4 of the word, so bits 8 .. 31 still hold
    // it) and takes its fields 8 bits lower
    uint32_t tail = 0;
    auto issue = [&](int g0, int c, bool refill) {
        const uint32_t voff = (uint32_t(5 * (n2 * g0 - c + t)) >> 2) - tail;
        if (refill) {
            const uint32_t v0 = voff - uint32_t((T - 1) * row_bytes);      // row g0-T+1, in the region
            gptr8 rp = (gptr8)rs;
#pragma unroll
            for (int k = 0; k < T - 1; ++k) {
                asm volatile("" : "+s"(rp));
                X0[k] = __builtin_bit_cast(float, load_u32u(rp, v0));
                rp += row_bytes;
            }
        }
        gptr8 rp = (gptr8)rs;
#pragma unroll
        for (int r = 0; r < G; ++r) {
            asm volatile("" : "+s"(rp));
            // rows past the region's last one (only padded outputs use them)
            // read that last row
            W[r] = load_u32u(rp, voff);
            if (g0 + r + 1 < mrows)
                rp += row_bytes;
        }
    };

    // a group's outputs are stored as soon as they are formed, behind the
    // next group's loads (one in-order counter covers both, so the wait for
    // those loads counts exactly G later stores: the stores are
    // unconditional, and outputs r >= the group's count take the scalar
    // offset DROP, beyond the buffer's record count, where the hardware
    // drops them: gfx950's range check of a raw buffer covers the scalar
    // offset too -- a store at vector offset 0 and scalar offset past the
    // record count writes nothing, tested inside a larger allocation)
    constexpr uint32_t DROP = 0x80000000u;

    // FRONT: rows row0 .. row0 + cnt - 1 (of g) from the tile, as described above
    auto front = [&](int row0, int cnt) {
        __syncthreads();                                      // the tile is written
        if (tid < 16 * G) {
            const int r = tid >> 4, gl = tid & 15;
            if (r < cnt) {
                float2 v[16];
#pragma unroll
                for (int q = 0; q < 16; ++q)
                    v[q] = fl[r][q][gl];
                Dft<16 + 0 * T>::run(v);                      // (dependent: Dft is complete by instantiation)
                const int gam = gbase + gl;
                const int64_t row = (int64_t(s) * M + row0 + r) * (n2 / 2);
                const float2 *tw = twf + int64_t(gam) * 16;
#pragma unroll
                for (int d = 0; d < 16; ++d) {
                    const float2 y = d == 0 ? v[0] : cmul(v[d], tw[d]);
                    if constexpr (GM == G_F16)
                        static_cast<uint32_t *>(g)[row + gam + gpt * d] = f16_pair(y);
                    else
                        static_cast<float2 *>(g)[row + gam + gpt * d] = y;
                }
            }
        }
        __syncthreads();                                      // the tile is read
    };

    for (int sa = m0; sa < mend; sa += FIR_SEG) {
        const int se = min(sa + FIR_SEG, mend);
        __syncthreads();                                      // the last segment's table is read
        for (int i = tid; i < se - sa; i += FIR_THREADS) {
            int c;
            double tau;
            s_c[i] = split_delay(ds[sa + i - moff], D, c, tau) ? c : -1;
        }
        __syncthreads();

        int m = sa;
        while (m < se) {
            const int c = __builtin_amdgcn_readfirstlane(s_c[m - sa]);
            if (c < 0 || int64_t(n2) * (m - T + 1) - c + t_blk < 0) {
                // general path for spectrum m, both columns
                int i = n2 * (m - T + 1) - max(c, 0) + t;
                float a0 = 0.f, a1 = 0.f;
#pragma unroll
                for (int j = 0; j < T; ++j) {
                    asm volatile("" : "+v"(i));
                    a0 = fmaf(float(sample_at(rs, hs, i, H)), h[j].x, a0);
                    a1 = fmaf(float(sample_at(rs, hs, i + 1, H)), h[j].y, a1);
                    i += n2;
                }
                if constexpr (FRONT) {
                    fl[0][tid >> 4][tid & 15] = c >= 0 ? make_float2(a0, a1) : make_float2(0.f, 0.f);
                    front(m - moff, 1);
                } else {
                    store_g2<GM>(c >= 0 ? a0 : 0.f, c >= 0 ? a1 : 0.f, rg, t_bytes, uint32_t((m - moff) * n2) * ES);
                }
                c_cur = -1;
                ++m;
                continue;
            }
            int send = m;
            for (;;) {
                const int ix = send - sa + lane;
                const int v = ix < se - sa ? s_c[ix] : -2;
                const uint64_t other = ~__builtin_amdgcn_ballot_w64(v == c);
                if (other) {
                    send += int(__builtin_ctzll(other));
                    break;
                }
                send += 64;
            }
            tail = (uint32_t(5 * (n2 * (mrows - 1) - c + t)) >> 2) + 4u > region_bytes ? 1u : 0u;
            const bool refill = c != c_cur;
            issue(m, c, refill);
            // the first sample's field in the byte-swapped word
            const uint32_t lo = 22u - ((uint32_t(t - c) & 3u) << 1) - 8u * tail;
            if (refill) {
#pragma unroll
                for (int i = 0; i < T - 1; ++i) {
                    const int32_t be = int32_t(__builtin_amdgcn_perm(0u, __builtin_bit_cast(uint32_t, X0[i]), 0x00010203u));
                    X0[i] = float(int32_t(__builtin_amdgcn_sbfe(be, lo, 10u)));
                    X1[i] = float(int32_t(__builtin_amdgcn_sbfe(be, lo - 10u, 10u)));
                }
            }
            for (int g0 = m;; g0 += G) {
                float Y0[G], Y1[G];
#pragma unroll
                for (int r = 0; r < G; ++r) {
                    const int32_t be = int32_t(__builtin_amdgcn_perm(0u, W[r], 0x00010203u));
                    Y0[r] = float(int32_t(__builtin_amdgcn_sbfe(be, lo, 10u)));
                    Y1[r] = float(int32_t(__builtin_amdgcn_sbfe(be, lo - 10u, 10u)));
                }
                const bool ahead = g0 + G < send;
                issue(ahead ? g0 + G : g0, c, false);
                __builtin_amdgcn_sched_barrier(0);            // keep the loads ahead of the arithmetic
                const int cnt = min(G, send - g0);
                const uint32_t soff = uint32_t((g0 - moff) * n2) * ES;
#pragma unroll
                for (int r = 0; r < G; ++r) {
                    float a0 = 0.f, a1 = 0.f;
#pragma unroll
                    for (int j = 0; j < T; ++j) {
                        a0 = fmaf(j + r < T - 1 ? X0[j + r] : Y0[j + r - (T - 1)], h[j].x, a0);
                        a1 = fmaf(j + r < T - 1 ? X1[j + r] : Y1[j + r - (T - 1)], h[j].y, a1);
                    }
                    if constexpr (FRONT)
                        fl[r][tid >> 4][tid & 15] = make_float2(a0, a1);
                    else
                        store_g2<GM>(a0, a1, rg, t_bytes, r < cnt ? soff + uint32_t(r * n2) * ES : DROP);
                }
                if constexpr (FRONT)
                    front(g0 - moff, cnt);
                // the window's last T-1 rows become the older rows of the next group
#pragma unroll
                for (int i = 0; i < T - 1; ++i) {
                    X0[i] = i + G < T - 1 ? X0[i + G] : Y0[i + G - (T - 1)];
                    X1[i] = i + G < T - 1 ? X1[i + G] : Y1[i + G - (T - 1)];
                }
                if (!ahead)
                    break;
            }
            c_cur = (send - m) % G == 0 ? c : -1;
            m = send;
        }
    }
}

template <int T, int GM, bool FRONT = false>
__global__ __launch_bounds__(FIR_THREADS, FRONT ? 2 : FIR_WG_PER_CU(T)) void fir_kernel(
    const uint8_t *__restrict__ raw, int64_t raw_stride,
    const uint8_t *__restrict__ hist, int64_t hist_stride, int H,
    const float *__restrict__ taps, const double *__restrict__ delays,
    void *__restrict__ g, int n2, int M, int D, int R, int colblocks, int runs, int mb, int me,
    int moff, int mrows, const float2 *__restrict__ twf)
{
    __shared__ int s_c[FIR_SEG];
    __shared__ float2 fl[FRONT ? fir_group(T) : 1][16][17];
    fir_block<T, GM, FRONT>(xcd_logical(blockIdx.x, gridDim.x), s_c, raw, raw_stride, hist, hist_stride, H, taps,
                            delays, g, n2, M, D, R, colblocks, runs, mb, me, moff, mrows, fl, twf);
}

// The seam of a call for the FIR: per stream, dst = [zero bytes | the
// history (hist_bytes) | the chunk's first head_bytes], as 32-bit words (all
// sizes and offsets are multiples of 4 bytes).
__global__ void seam_stage_kernel(uint32_t *__restrict__ dst, int64_t dst_words,
                                  const uint32_t *__restrict__ hist, int64_t hist_words,
                                  const uint32_t *__restrict__ raw, int64_t raw_words,
                                  int64_t zero_words, int64_t head_words, int streams)
{
    const int64_t total = dst_words * streams;
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
         e += int64_t(gridDim.x) * blockDim.x) {
        const int64_t s = e / dst_words, i = e % dst_words;
        uint32_t v = 0u;
        if (i >= zero_words && i < zero_words + hist_words)
            v = hist[s * hist_words + (i - zero_words)];
        else if (i >= zero_words + hist_words && i < zero_words + hist_words + head_words)
            v = raw[s * raw_words + (i - zero_words - hist_words)];
        dst[e] = v;
    }
}

// ---------------------------------------------------------------------------
// FFT building blocks: in-register DFTs of size 2, 4, 8, 16 (forward,
// exp(-2 pi i m k / R)), natural order in and out.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void dft2(float2 &a, float2 &b)
{
    const float2 t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

__device__ __forceinline__ void dft4(float2 &x0, float2 &x1, float2 &x2, float2 &x3)
{
    const float2 s02 = cadd(x0, x2), d02 = csub(x0, x2);
    const float2 s13 = cadd(x1, x3), d13 = cmul_mi(csub(x1, x3));
    x0 = cadd(s02, s13);
    x2 = csub(s02, s13);
    x1 = cadd(d02, d13);
    x3 = csub(d02, d13);
}

constexpr float kR2 = 0.70710678118654752440f;     // cos(pi/4)
constexpr float kC8 = 0.92387953251128675613f;     // cos(pi/8)
constexpr float kS8 = 0.38268343236508977173f;     // sin(pi/8)

template <int R> struct Dft;

template <> struct Dft<2> {
    __device__ static void run(float2 *x) { dft2(x[0], x[1]); }
};

template <> struct Dft<4> {
    __device__ static void run(float2 *x) { dft4(x[0], x[1], x[2], x[3]); }
};

// 8 = 4 x 2: m = 2 m1 + m2, k = k1 + 4 k2
template <> struct Dft<8> {
    __device__ static void run(float2 *x)
    {
        float2 e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
        float2 o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
        dft4(e0, e1, e2, e3);
        dft4(o0, o1, o2, o3);
        // twiddle W8^k1 on the odd half
        o1 = make_float2(kR2 * (o1.x + o1.y), kR2 * (o1.y - o1.x));
        o2 = cmul_mi(o2);
        o3 = make_float2(kR2 * (o3.y - o3.x), -kR2 * (o3.x + o3.y));
        x[0] = cadd(e0, o0); x[4] = csub(e0, o0);
        x[1] = cadd(e1, o1); x[5] = csub(e1, o1);
        x[2] = cadd(e2, o2); x[6] = csub(e2, o2);
        x[3] = cadd(e3, o3); x[7] = csub(e3, o3);
    }
};

// 16 = 4 x 4: m = 4 m1 + m2, k = k1 + 4 k2
template <> struct Dft<16> {
    __device__ static void run(float2 *x)
    {
#pragma unroll
        for (int m2 = 0; m2 < 4; ++m2)
            dft4(x[m2], x[m2 + 4], x[m2 + 8], x[m2 + 12]);     // -> y[m2][k1] at x[m2 + 4 k1]
        // twiddles W16^(m2 k1)
        const float2 w1 = make_float2(kC8, -kS8), w2 = make_float2(kR2, -kR2), w3 = make_float2(kS8, -kC8);
        x[5] = cmul(x[5], w1);                       // m2=1,k1=1
        x[9] = cmul(x[9], w2);                       // m2=1,k1=2
        x[13] = cmul(x[13], w3);                     // m2=1,k1=3
        x[6] = cmul(x[6], w2);                       // m2=2,k1=1
        x[10] = cmul_mi(x[10]);                      // m2=2,k1=2 (W^4)
        x[14] = cmul(x[14], make_float2(-kR2, -kR2));    // m2=2,k1=3 (W^6)
        x[7] = cmul(x[7], w3);                       // m2=3,k1=1 (W^3)
        x[11] = cmul(x[11], make_float2(-kR2, -kR2));    // m2=3,k1=2 (W^6)
        x[15] = cmul(x[15], make_float2(-kC8, kS8));     // m2=3,k1=3 (W^9)
        float2 y[16];
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            float2 a = x[4 * k1], b = x[4 * k1 + 1], c = x[4 * k1 + 2], d = x[4 * k1 + 3];
            dft4(a, b, c, d);                        // over m2 -> k2
            y[k1] = a; y[k1 + 4] = b; y[k1 + 8] = c; y[k1 + 12] = d;
        }
#pragma unroll
        for (int i = 0; i < 16; ++i)
            x[i] = y[i];
    }
};

// ---------------------------------------------------------------------------
// FFT plans: radices in execution order; n = product.  Threads per
// polarization = n/16, each owning 16 points (16/R butterflies per pass).
// ---------------------------------------------------------------------------

template <int N> struct Plan;
template <> struct Plan<256>  { static constexpr int P = 2; static constexpr int R[4] = {16, 16, 1, 1}; };
template <> struct Plan<512>  { static constexpr int P = 3; static constexpr int R[4] = {16, 16, 2, 1}; };
template <> struct Plan<1024> { static constexpr int P = 3; static constexpr int R[4] = {16, 16, 4, 1}; };
template <> struct Plan<2048> { static constexpr int P = 3; static constexpr int R[4] = {16, 16, 8, 1}; };
template <> struct Plan<4096> { static constexpr int P = 3; static constexpr int R[4] = {16, 16, 16, 1}; };
template <> struct Plan<8192> { static constexpr int P = 4; static constexpr int R[4] = {16, 16, 16, 2}; };

// Host and device agree on the twiddle-table layout: for each pass p with
// L_p = R_0 ... R_{p-1} > 1, a block [R_p - 1][L_p] of exp(-2 pi i j q / (L_p R_p))
// (q-major, so the lanes of a wave, which hold consecutive j, read one
// contiguous segment per q).
template <int N>
__host__ __device__ constexpr int tw_offset(int p)
{
    int off = 0, L = 1;
    for (int i = 0; i < p; ++i) {
        if (L > 1)
            off += L * (Plan<N>::R[i] - 1);
        L *= Plan<N>::R[i];
    }
    return off;
}

template <int N>
__host__ __device__ constexpr int tw_L(int p)
{
    int L = 1;
    for (int i = 0; i < p; ++i)
        L *= Plan<N>::R[i];
    return L;
}

// LDS layout of one polarization's n points: one float2 of padding after
// every 16, so that the radix-16 pass with L = 1 (lane stride 16 elements)
// and the L = 16 pass (groups of 16 at stride 256) hit distinct banks.
constexpr int lds_pad(int i) { return i + (i >> 4); }
template <int N> constexpr int lds_len() { return N + N / 16; }

// One Stockham pass (radix R, L = product of earlier radices) over one
// polarization's n points held in LDS:
//   butterfly b: inputs z[b + q n/R], twiddle exp(-2 pi i j q/(L R)) with
//   j = b mod L, R-point DFT, outputs to (b - j) R + j + r L.
// TWL (kernels whose vector memory instructions, not only their arithmetic,
// bound them): the L = 16 pass reads its 240 twiddles from the LDS copy
// `tws`, and passes with L > 16 and R = 8 or 16 load w^1 .. w^4, w^8 and w^12
// (w = exp(-2 pi i j/(L R))) and form the other powers w^(4a + b) = w^4a w^b,
// one product each.
template <int N, int R, int L, bool TWL>
__device__ __forceinline__ void fft_pass(float2 *__restrict__ buf, int tp, const float2 *__restrict__ tw,
                                         const float2 *__restrict__ tws)
{
    constexpr int NB = N / R;              // butterflies per polarization
    constexpr int NTP = N / 16;            // threads per polarization
    constexpr int PER = NB / NTP;          // butterflies per thread
    float2 v[PER][R];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int b = tp + u * NTP;
#pragma unroll
        for (int q = 0; q < R; ++q)
            v[u][q] = buf[lds_pad(b + q * NB)];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int b = tp + u * NTP;
        const int j = b % L;
        if constexpr (TWL && L == 16) {
#pragma unroll
            for (int q = 1; q < R; ++q)
                v[u][q] = cmul(v[u][q], tws[(q - 1) * L + j]);
        } else if constexpr (TWL && R > 4) {
            // w^1 .. w^4 and w^8, w^12 loaded; w^(4a + b) = w^4a w^b
            float2 wq[R];
#pragma unroll
            for (int q = 1; q <= 4; ++q)
                wq[q] = tw[(q - 1) * L + j];
            if constexpr (R > 8) {
                wq[8] = tw[7 * L + j];
                wq[12] = tw[11 * L + j];
            }
#pragma unroll
            for (int q = 5; q < R; ++q)
                if (q % 4 != 0)
                    wq[q] = cmul(wq[q - q % 4], wq[q % 4]);
#pragma unroll
            for (int q = 1; q < R; ++q)
                v[u][q] = cmul(v[u][q], wq[q]);
        } else {
#pragma unroll
            for (int q = 1; q < R; ++q)
                v[u][q] = cmul(v[u][q], tw[(q - 1) * L + j]);
        }
        Dft<R>::run(v[u]);
        const int base = (b - j) * R + j;
#pragma unroll
        for (int r = 0; r < R; ++r)
            buf[lds_pad(base + r * L)] = v[u][r];
    }
    __syncthreads();
}

// Passes 1.. of the plan (pass 0, radix 16 with L = 1, is done by the caller
// on register-held input).  Every plan's pass 1 is radix 16 with L = 16: its
// twiddle block is the table's first 240 entries.
constexpr int TW_PASS1 = 15 * 16;

template <int N, int P, bool TWL = false>
__device__ __forceinline__ void fft_rest(float2 *buf, int tp, const float2 *tw_all, const float2 *tws = nullptr)
{
    if constexpr (P < Plan<N>::P) {
        constexpr int R = Plan<N>::R[P];
        constexpr int L = tw_L<N>(P);
        static_assert(P != 1 || (R == 16 && L == 16 && tw_offset<N>(1) == 0), "pass 1 is radix 16, L = 16");
        fft_pass<N, R, L, TWL>(buf, tp, tw_all + tw_offset<N>(P), tws);
        fft_rest<N, P + 1, TWL>(buf, tp, tw_all, tws);
    }
}

// Copy of the pass-1 twiddles into LDS (read after the caller's next barrier).
__device__ __forceinline__ void load_tw_pass1(float2 *__restrict__ tws, const float2 *__restrict__ tw_all,
                                              int tid, int nt)
{
    for (int i = tid; i < TW_PASS1; i += nt)
        tws[i] = tw_all[i];
}

// ---------------------------------------------------------------------------
// Kernel 2: FFT + real-FFT untangle + fine delay/phase + gain + quantise.
// One workgroup of n/16 threads per (antenna, polarization, spectrum), 16
// points per thread: radix-16 Stockham passes in LDS, the first one on the
// registers loaded from g.  Each thread then finishes channel pairs
// (2j, 2j+1), j = tid + (n/16) i.  In int8 mode the spectrum's n (re, im)
// byte pairs go contiguously into a spectrum-major staging buffer
// [A][2][M][n][2] (kernel 3 turns it into heaps); in prequant mode Y is
// written instead.
// ---------------------------------------------------------------------------

enum { OUT_INT8 = 0, OUT_PREQUANT = 1, OUT_REG = 3 };   // OUT_REG: the int8 dwords stay in registers

// Four values to four int8 in one dword (byte i = value i): saturate to
// [-127, 127], round half to even.  Clamping first gives the same result as
// rounding first (the bounds are integers).  Adding 1.5 * 2^23 rounds the
// clamped value to an integer r in the float's own rounding (to nearest,
// ties to even: the sum's unit in the last place is 1) and leaves
// 0x400000 + r in its mantissa, whose low byte is r in two's complement.
// Finite inputs only.
__device__ __forceinline__ uint32_t quant4(float a, float b, float c, float d)
{
    constexpr float kRound = 12582912.0f;                 // 1.5 * 2^23
    const uint32_t ya = __builtin_bit_cast(uint32_t, __builtin_amdgcn_fmed3f(a, -127.f, 127.f) + kRound);
    const uint32_t yb = __builtin_bit_cast(uint32_t, __builtin_amdgcn_fmed3f(b, -127.f, 127.f) + kRound);
    const uint32_t yc = __builtin_bit_cast(uint32_t, __builtin_amdgcn_fmed3f(c, -127.f, 127.f) + kRound);
    const uint32_t yd = __builtin_bit_cast(uint32_t, __builtin_amdgcn_fmed3f(d, -127.f, 127.f) + kRound);
    // byte selectors 0-3 take the second operand, 4-7 the first, 0x0c gives 0
    const uint32_t lo = __builtin_amdgcn_perm(yb, ya, 0x0c0c0400u);       // (a, b, 0, 0)
    const uint32_t hi = __builtin_amdgcn_perm(yd, yc, 0x04000c0cu);       // (0, 0, c, d)
    return lo | hi;
}

// Per-spectrum phase tables: exp(i(phi - pi k tau / n)) = ph_hi[k >> 6] *
// ph_lo[k & 63] / lo_scale.  Arguments in revolutions, reduced in float64,
// sin/cos in float32.  ph_lo also carries `lo_scale` (a power of two: the
// factor 1/2 of the real-FFT untangle and any FFT stage scaling).
template <int N, int NT>
__device__ __forceinline__ void phase_tables(float2 *ph_hi, float2 *ph_lo, double phi, double tau,
                                             float lo_scale, int tid)
{
    constexpr int NH = N / 64;
    constexpr double inv_two_pi = 0.15915494309189533577;
    constexpr double inv_two_n = 0.5 / N;          // exact: N is a power of two
    const double tau_rev = tau * inv_two_n;
    const double phi_rev = phi * inv_two_pi;
    for (int i = tid; i < NH + 64; i += NT) {
        double rev = i < NH ? phi_rev - double(64 * i) * tau_rev : -double(i - NH) * tau_rev;
        rev -= rint(rev);
        float sn, cs;
        sincospif(float(2.0 * rev), &sn, &cs);
        if (i < NH)
            ph_hi[i] = make_float2(cs, sn);
        else
            ph_lo[i - NH] = make_float2(lo_scale * cs, lo_scale * sn);
    }
}

// Steps 3b-6 on one polarization's n-point complex FFT Z held in LDS (natural
// order, lds_pad layout): real-FFT untangle, phase, gain, then either the
// int8 pair store or the pre-quantisation store.  Thread tid finishes channel
// pairs (2j, 2j+1), j = tid + NT i.  The int8 pairs are stored through the
// caches: the corner turn reads them next.
template <int N, int NT, int MODE, bool UNT_CALC = false>
__device__ __forceinline__ void post_spectrum(const float2 *__restrict__ buf, const float2 *ph_hi,
                                              const float2 *ph_lo, const float2 *__restrict__ untangle,
                                              const float2 *__restrict__ gn, bool ok, int64_t sp, int tid,
                                              uint32_t *__restrict__ spec8, float2 *__restrict__ y_out,
                                              bool store = true, uint32_t *qreg = nullptr)
{
    // channel k = k0 + S i with k0 = 2 tid + e: the padded LDS offsets of k
    // and n - k, the coarse phase index and the table offsets all step by
    // constants with i (S is a multiple of 16; of 64 from n = 512 up)
    constexpr int S = 2 * NT;
    constexpr int SP = S + S / 16;
    int pk[2], pm[2];
    float2 lo[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int k0 = 2 * tid + e;
        pk[e] = lds_pad(k0);
        pm[e] = lds_pad(N - k0);
        if constexpr (S % 64 == 0)
            lo[e] = ph_lo[k0 & 63];
    }
    // the per-channel constants (untangle twiddle, gain) come from L2: issue
    // all of this thread's loads before the first use, so their latencies
    // overlap instead of adding up channel by channel
    constexpr int P = N / 2 / NT;
    float4 wt[P], gt[P];
    if constexpr (UNT_CALC) {
        // (the matrix-core kernels, bound by their vector memory
        // instructions) the untangle twiddles w_k = exp(-i pi k / n) of
        // channels 2 tid + e + S i are the loaded w_{2 tid + e} times the
        // table's w_{S i}, whose index is the same in every lane (a scalar
        // load).  The product's extra rounding shows at the mirror channel of
        // a strong tone, where the untangle subtracts two terms of the tone's
        // size: there it reaches 1e-5 of the spectrum's rms, which the FP32
        // kernels' bound does not leave room for (they load the table).
        const float4 w01 = reinterpret_cast<const float4 *>(untangle)[tid];
        const float2 w0 = make_float2(w01.x, w01.y), w1 = make_float2(w01.z, w01.w);
        wt[0] = w01;
#pragma unroll
        for (int i = 1; i < P; ++i) {
            const float2 c = untangle[S * i];
            const float2 a = cmul(w0, c), b = cmul(w1, c);
            wt[i] = make_float4(a.x, a.y, b.x, b.y);
        }
    }
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const int j = tid + NT * i;
        if constexpr (!UNT_CALC)
            wt[i] = reinterpret_cast<const float4 *>(untangle)[j];
        gt[i] = reinterpret_cast<const float4 *>(gn)[j];
    }
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const int j = tid + NT * i;
        float2 Y[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int k = 2 * j + e;
            const float2 zk = buf[pk[e] + SP * i];
            // n - k, except k = 0, whose partner is itself
            const float2 zm = buf[(i == 0 && k == 0) ? 0 : pm[e] - SP * i];
            const float2 w = e == 0 ? make_float2(wt[i].x, wt[i].y) : make_float2(wt[i].z, wt[i].w);
            const float2 gk = e == 0 ? make_float2(gt[i].x, gt[i].y) : make_float2(gt[i].z, gt[i].w);
            // 2E = Z[k] + conj Z[n-k], 2O = (Z[k] - conj Z[n-k]) / i, 2X = 2E + w 2O
            const float2 E2 = make_float2(zk.x + zm.x, zk.y - zm.y);
            const float2 O2 = make_float2(zk.y + zm.y, zm.x - zk.x);
            const float2 X2 = cadd(E2, cmul(w, O2));                   // w = exp(-i pi k / n)
            const float2 l = (S % 64 == 0) ? lo[e] : ph_lo[k & 63];
            const float2 rot = cmul(ph_hi[k >> 6], l);                 // includes 1/2
            Y[e] = ok ? cmul(gk, cmul(rot, X2)) : make_float2(0.f, 0.f);
        }
        if (!store) {
        } else if (MODE == OUT_REG) {
            qreg[i] = quant4(Y[0].x, Y[0].y, Y[1].x, Y[1].y);
        } else if (MODE == OUT_PREQUANT) {
            reinterpret_cast<float4 *>(y_out + sp * N)[j] = make_float4(Y[0].x, Y[0].y, Y[1].x, Y[1].y);
        } else {
            spec8[sp * (N / 2) + j] = quant4(Y[0].x, Y[0].y, Y[1].x, Y[1].y);
        }
    }
}

// The body of kernel 2 for one work item ((a (me - mb) + F - mb) * 2 + p:
// both pols of a spectrum adjacent) by threads tid < n/16, with LDS buf
// (lds_len<N>), ph_hi (max(N/64, 1)) and ph_lo (64).  An item that is not
// `valid` runs the same arithmetic (and barriers) on item 0 and stores
// nothing.
template <int N, int MODE>
__device__ __forceinline__ void fft_post_block(
    int item, bool valid, int tid, float2 *__restrict__ buf, float2 *__restrict__ ph_hi,
    float2 *__restrict__ ph_lo, float2 *__restrict__ tws,
    const float *__restrict__ g, const double *__restrict__ delays,
    const double *__restrict__ phases, const float2 *__restrict__ gains,
    const float2 *__restrict__ tw_all, const float2 *__restrict__ untangle,
    uint32_t *__restrict__ spec8, float2 *__restrict__ y_out, int *__restrict__ status,
    int M, int D, int mb, int me)
{
    static_assert(Plan<N>::R[0] == 16, "plans start with a radix-16 pass");
    constexpr int NT = N / 16;             // threads, 16 points each
    if (!valid)
        item = 0;
    const int p = item & 1;
    const int af = item >> 1;
    const int a = af / (me - mb);
    const int F = mb + af % (me - mb);
    const int64_t sp = (int64_t(a) * 2 + p) * M + F;          // stream spectrum

    // z[m] = g[2m] + i g[2m+1]
    const float2 *src = reinterpret_cast<const float2 *>(g) + sp * N;
    float2 v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q)
        v[q] = load_nt(src + tid + q * NT);

    int c;
    double tau;
    const bool ok = split_delay(delays[sp], D, c, tau);
    if (valid && !ok && tid == 0)
        atomicOr(status, 1);
    phase_tables<N, NT>(ph_hi, ph_lo, phases[sp], tau, 0.5f, tid);
    load_tw_pass1(tws, tw_all, tid, NT);

    // forward n-point complex FFT: pass 0 in registers, the rest in LDS
    Dft<16>::run(v);
#pragma unroll
    for (int r = 0; r < 16; ++r)
        buf[lds_pad(tid * 16 + r)] = v[r];
    __syncthreads();
    fft_rest<N, 1, true>(buf, tid, tw_all, tws);

    post_spectrum<N, NT, MODE>(buf, ph_hi, ph_lo, untangle, gains + (int64_t(a) * 2 + p) * N, ok, sp,
                               tid, spec8, y_out, valid);
}

template <int N, int MODE>
__global__ __launch_bounds__(N / 16, (N / 16 >= 256 ? 4 : 1)) void fft_post_kernel(
    const float *__restrict__ g, const double *__restrict__ delays,
    const double *__restrict__ phases, const float2 *__restrict__ gains,
    const float2 *__restrict__ tw_all, const float2 *__restrict__ untangle,
    uint32_t *__restrict__ spec8, float2 *__restrict__ y_out, int *__restrict__ status,
    int M, int D, int mb, int me)
{
    constexpr int NH = N / 64;             // coarse phase-table entries (k >> 6)
    __shared__ float2 buf[lds_len<N>()];
    __shared__ float2 ph_hi[NH < 1 ? 1 : NH];
    __shared__ float2 ph_lo[64];
    __shared__ float2 tws[TW_PASS1];
    fft_post_block<N, MODE>(xcd_logical(blockIdx.x, gridDim.x), true, threadIdx.x, buf, ph_hi, ph_lo, tws, g,
                            delays, phases, gains, tw_all, untangle, spec8, y_out, status, M, D, mb, me);
}

// The int8 dwords q[2 f + p][i] (spectrum F0 + f, pol p; channels 2j, 2j+1,
// j = tid + NT i) of antenna a to their places in the heaps
// [A][M/S][n][S][2][2]: channel k's dword for one spectrum is (re, im) of pol
// 0, then of pol 1, and its SPW spectra are contiguous (F0 is a multiple of
// SPW, and SPW = 2 needs S even).
template <int N, int NT, int SPW, int P>
__device__ __forceinline__ void heap_store(const uint32_t (&q)[2 * SPW][P], int8_t *__restrict__ out, int a, int M,
                                           int S, int F0, int tid)
{
    uint32_t *o = reinterpret_cast<uint32_t *>(out) + (int64_t(a) * (M / S) + F0 / S) * N * S + F0 % S;
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const int j = tid + NT * i;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const uint32_t sel = e == 0 ? 0x05040100u : 0x07060302u;
            uint32_t w[SPW];
#pragma unroll
            for (int f = 0; f < SPW; ++f)
                w[f] = __builtin_amdgcn_perm(q[2 * f + 1][i], q[2 * f][i], sel);
            uint32_t *dst = o + int64_t(2 * j + e) * S;
            if constexpr (SPW == 2)
                *reinterpret_cast<uint2 *>(dst) = make_uint2(w[0], w[1]);
            else
                *dst = w[0];
        }
    }
}

// ---------------------------------------------------------------------------
// Kernel 2H: kernel 2 with the corner turn folded in (int8 output, n <= 8192).
// One workgroup per (antenna, run of SPW consecutive spectra F0 ..): it
// transforms and finishes the two polarizations of each spectrum in turn,
// keeping each one's int8 pairs in registers, then writes every channel's
// SPW spectra x 2 pols x (re, im) bytes straight to their place in the heap,
// [A][M/S][n][S][2][2]: 4 SPW contiguous bytes per channel.  A wave's store
// touches 64 lines, and consecutive runs of one antenna sit on one XCD, so
// that XCD's L2 merges the runs' pieces of each line before they go to HBM.
// SPW = 2 needs S even (a run never straddles heaps).
// ---------------------------------------------------------------------------

template <int N, int SPW>
__global__ __launch_bounds__(N / 16, (N / 16 >= 256 ? 4 : 1)) void fft_post_heap_kernel(
    const float *__restrict__ g, const double *__restrict__ delays,
    const double *__restrict__ phases, const float2 *__restrict__ gains,
    const float2 *__restrict__ tw_all, const float2 *__restrict__ untangle,
    int8_t *__restrict__ out, int *__restrict__ status, int M, int D, int S)
{
    constexpr int NT = N / 16;             // threads, 16 points each
    constexpr int NH = N / 64;
    constexpr int P = N / 2 / NT;          // channel pairs per thread
    __shared__ float2 buf[lds_len<N>()];
    __shared__ float2 ph_hi[NH < 1 ? 1 : NH];
    __shared__ float2 ph_lo[64];
    __shared__ float2 tws[TW_PASS1];
    const int runs = M / SPW;
    const int item = xcd_logical(blockIdx.x, gridDim.x);
    const int a = item / runs;
    const int F0 = (item % runs) * SPW;

    // q[2 f + p]: the int8 dwords of spectrum F0 + f, pol p.  The loop is
    // not unrolled (unrolled, the compiler hoists every transform's loads to
    // the top and spills); each pass shifts its result in at the end.
    constexpr int Q = 2 * SPW;
    uint32_t q[Q][P];
#pragma unroll
    for (int u = 0; u < Q; ++u)
#pragma unroll
        for (int i = 0; i < P; ++i)
            q[u][i] = 0u;
    load_tw_pass1(tws, tw_all, int(threadIdx.x), NT);      // read after the first pass's barrier
#pragma unroll 1
    for (int fp = 0; fp < Q; ++fp) {
        const int f = fp >> 1, p = fp & 1;
        // a fresh copy of the thread index and table bases per pass, so that
        // the addresses and table loads derived from them are not hoisted
        // out of the loop (and held across it, in registers it does not have)
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const float2 *tw = tw_all, *ut = untangle;
        asm volatile("" : "+s"(tw), "+s"(ut));
        const int64_t sp = (int64_t(a) * 2 + p) * M + F0 + f;
        const float2 *src = reinterpret_cast<const float2 *>(g) + sp * N;
        float2 v[16];
#pragma unroll
        for (int r = 0; r < 16; ++r)
            v[r] = load_nt(src + tid + r * NT);
        int c;
        double tau;
        const bool ok = split_delay(delays[sp], D, c, tau);
        if (!ok && tid == 0)
            atomicOr(status, 1);
        if (fp > 0)
            __syncthreads();               // the previous pass's readers are done with LDS
        phase_tables<N, NT>(ph_hi, ph_lo, phases[sp], tau, 0.5f, tid);
        Dft<16>::run(v);
#pragma unroll
        for (int r = 0; r < 16; ++r)
            buf[lds_pad(tid * 16 + r)] = v[r];
        __syncthreads();
        fft_rest<N, 1, true>(buf, tid, tw, tws);
        uint32_t qn[P];
        post_spectrum<N, NT, OUT_REG>(buf, ph_hi, ph_lo, ut, gains + (int64_t(a) * 2 + p) * N, ok, sp,
                                      tid, nullptr, nullptr, true, qn);
#pragma unroll
        for (int i = 0; i < P; ++i) {
#pragma unroll
            for (int u = 0; u + 1 < Q; ++u)
                q[u][i] = q[u + 1][i];
            q[Q - 1][i] = qn[i];
        }
    }

    heap_store<N, NT, SPW, P>(q, out, a, M, S, F0, int(threadIdx.x));
}

// ---------------------------------------------------------------------------
// Kernel 1F (n <= 4096, FP32): the whole path of one stream in one kernel --
// unpack, coarse delay and the FIR of Eq. (1) straight into LDS, then the
// n-point complex FFT there, the untangle, phase, gain and quantisation of
// kernel 2.  No filtered sample leaves the workgroup.
//
// Workgroup = one stream (antenna, pol) and a run of steps of PF_S = 4
// consecutive spectra F0 .. F0+3.  Thread b (of n/4) owns the column pairs
// m = b + (n/4) q, q < 4 (z[m] = g[2m] + i g[2m+1]) of all four spectra.
// When the step's spectra share one coarse delay c, they read rows
// F0-T+1 .. F0+3 of those columns at offset -c, so each loaded pair of
// samples serves up to four outputs (T + 3 rows for 4 T products per
// column), and each column's taps, read from L2 once per step, serve the four
// spectra.  A pair of samples (20 bits) lies in the 4 bytes from byte
// floor(5 i / 4) of its first sample i: one unaligned dword load, a byte
// swap, two sign-extending bitfield extracts.  Steps whose spectra differ in
// delay, read rows before the call (the history seam) or have an invalid
// delay take a per-spectrum path.  The four spectra's z go to four LDS
// buffers; thread groups of n/16 then transform one spectrum each (radix-16
// Stockham passes) and finish its channels.
// ---------------------------------------------------------------------------

constexpr int PF_S = 4;                     // spectra per step

enum { OUT_G = 2 };                         // (besides OUT_INT8, OUT_PREQUANT) the FIR output g


// Radix-16 Stockham pass with L = 1 (no twiddles) over one polarization's n
// points in LDS: butterfly b reads z[b + q n/16], writes 16 b + r.
template <int N>
__device__ __forceinline__ void fft_pass0(float2 *__restrict__ buf, int tp)
{
    constexpr int NB = N / 16;
    float2 v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q)
        v[q] = buf[lds_pad(tp + q * NB)];
    __syncthreads();
    Dft<16>::run(v);
#pragma unroll
    for (int r = 0; r < 16; ++r)
        buf[lds_pad(tp * 16 + r)] = v[r];
    __syncthreads();
}

// taps (h[2m + 2n j], h[2m + 1 + 2n j]), j < T, of column pair m: a scalar
// row pointer plus one lane offset per load
template <int T, int N2>
__device__ __forceinline__ void load_tap_pairs(float2 (&h)[T], const float *taps, int m)
{
    typedef float v2f __attribute__((ext_vector_type(2)));
    typedef const v2f __attribute__((address_space(1))) *gptr_v2f;
    gptr8 tb = (gptr8)taps;
    const uint32_t off = uint32_t(m) * 8u;
#pragma unroll
    for (int j = 0; j < T; ++j) {
        asm volatile("" : "+s"(tb));
        const v2f v = *reinterpret_cast<gptr_v2f>(tb + off);
        h[j] = make_float2(v.x, v.y);
        tb += N2 * 4;
    }
}

template <int N, int T, int MODE>
__global__ __launch_bounds__(N / 4) void pfb_fused_kernel(
    const uint8_t *__restrict__ raw, int64_t raw_stride,
    const uint8_t *__restrict__ hist, int64_t hist_stride, int H,
    const float *__restrict__ taps, const double *__restrict__ delays,
    const double *__restrict__ phases, const float2 *__restrict__ gains,
    const float2 *__restrict__ tw_all, const float2 *__restrict__ untangle,
    uint32_t *__restrict__ spec8, float2 *__restrict__ y_out, float2 *__restrict__ g_out,
    int *__restrict__ status, int M, int D, int streams, int mb, int me)
{
    static_assert(Plan<N>::R[0] == 16, "plans start with a radix-16 pass");
    constexpr int NT = N / 4;               // threads: 4 column pairs each
    constexpr int NTP = N / 16;             // threads per spectrum in the FFT
    constexpr int NH = N / 64;
    constexpr int n2 = 2 * N;
    constexpr int row_bytes = n2 / 4 * 5;   // 2n packed samples
    constexpr int NR = T + PF_S - 1;        // rows of a step
    __shared__ float2 buf[PF_S][lds_len<N>()];
    __shared__ float2 ph_hi[PF_S][NH < 1 ? 1 : NH];
    __shared__ float2 ph_lo[PF_S][64];

    // Work units (stream, step) in stream-major order are split into eight
    // contiguous ranges, one per XCD (workgroup b runs on XCD b mod 8; the
    // grid is a multiple of 8).  The K workgroups of an XCD interleave their
    // range's steps (unit u0 + k, u0 + k + K, ...), so that at any time they
    // work on neighbouring steps of a stream and share its rows and the taps
    // in their L2.
    const int xcd = blockIdx.x & 7, k = blockIdx.x >> 3, K = gridDim.x >> 3;
    const int nsteps = (me - mb + PF_S - 1) / PF_S;
    const int64_t units = int64_t(streams) * nsteps;
    const int64_t u_begin = units * xcd / 8, u_end = units * (xcd + 1) / 8;
    const int tid = threadIdx.x;

    for (int64_t u = u_begin + k; u < u_end; u += K) {
        const int s = int(u / nsteps);                    // stream = 2 a + p
        const int step = int(u - int64_t(s) * nsteps);
        const int F0 = mb + PF_S * step;
        const uint8_t *rs = raw + int64_t(s) * raw_stride;
        const double *ds = delays + int64_t(s) * M;
        // lane values are derived afresh each step (hoisted out of the step
        // loop, their 64-bit addresses would not fit the registers)
        int ltid = tid;
        asm volatile("" : "+v"(ltid));
        const int fg = ltid / NTP, tp = ltid % NTP;
        // the step's delays (the same in every lane)
        int cf[PF_S];
        double tauf[PF_S];
        bool okf[PF_S], live[PF_S];
#pragma unroll
        for (int f = 0; f < PF_S; ++f) {
            live[f] = F0 + f < me;
            okf[f] = live[f] && split_delay(ds[F0 + f], D, cf[f], tauf[f]);
        }
        if (tid == 0) {
#pragma unroll
            for (int f = 0; f < PF_S; ++f)
                if (live[f] && !okf[f])
                    atomicOr(status, 1);
        }
        if (MODE != OUT_G && live[fg])
            phase_tables<N, NTP>(ph_hi[fg], ph_lo[fg], phases[int64_t(s) * M + F0 + fg], tauf[fg], 0.5f, tp);

        const int c = cf[0];
        bool fast = okf[0] && okf[1] && okf[2] && okf[3] && cf[1] == c && cf[2] == c && cf[3] == c
                    && int64_t(n2) * (F0 - T + 1) - c >= 0;
        if (fast) {
            // rows F0-T+1 .. F0+3 at delay c: c = 2n cr + cc, so the rows start
            // cr rows earlier and lane offsets keep cc (plus one row of
            // margin, so that they are never negative)
            const int cr = c / n2, cc = c - cr * n2;
            const gptr8 rp0 = (gptr8)rs + int64_t(F0 - T + 1 - cr - 1) * row_bytes;
            // the call's last row: a pair that does not need the fourth byte
            // from its first is read from one byte earlier, so that no load
            // passes the end of the chunk
            const bool tail = F0 + PF_S - 1 - cr == M - 1;
            auto lane_geo = [&](int q, uint32_t &off, uint32_t &lo0, uint32_t &shl) {
                const int u2 = 2 * (ltid + NT * q) - cc;          // first sample of the pair in its row
                const uint32_t ua = uint32_t(u2) & 3u;
                off = uint32_t(row_bytes + ((5 * u2) >> 2));
                lo0 = 22u - 2u * ua;                              // bit position of the first sample
                shl = tail && ua != 3u ? 1u : 0u;
            };
            auto load_rows = [&](int q, uint32_t (&w)[NR]) {
                uint32_t off, lo0, shl;
                lane_geo(q, off, lo0, shl);
                gptr8 rp = rp0;
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    asm volatile("" : "+s"(rp));
                    w[r] = load_u32u(rp, r == NR - 1 ? off - shl : off);
                    rp += row_bytes;
                }
            };
            // the rows of pair q + 1 are loaded while pair q is filtered
            uint32_t wn[NR];
            load_rows(0, wn);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = ltid + NT * q;
                uint32_t w[NR];
#pragma unroll
                for (int r = 0; r < NR; ++r)
                    w[r] = wn[r];
                if (q + 1 < 4)
                    load_rows(q + 1, wn);
                float2 h[T];
                load_tap_pairs<T, n2>(h, taps, m);
                uint32_t off, lo0, shl;
                lane_geo(q, off, lo0, shl);
                float x0[NR], x1[NR];
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const uint32_t lo = r == NR - 1 ? lo0 - 8u * shl : lo0;
                    const int32_t be = int32_t(__builtin_amdgcn_perm(0u, w[r], 0x00010203u));
                    x0[r] = float(int32_t(__builtin_amdgcn_sbfe(be, lo, 10u)));
                    x1[r] = float(int32_t(__builtin_amdgcn_sbfe(be, lo - 10u, 10u)));
                }
#pragma unroll
                for (int f = 0; f < PF_S; ++f) {
                    float a0 = 0.f, a1 = 0.f;
#pragma unroll
                    for (int j = 0; j < T; ++j) {
                        a0 = fmaf(x0[f + j], h[j].x, a0);
                        a1 = fmaf(x1[f + j], h[j].y, a1);
                    }
                    if (MODE == OUT_G)
                        g_out[(int64_t(s) * M + F0 + f) * N + m] = make_float2(a0, a1);
                    else
                        buf[f][lds_pad(m)] = make_float2(a0, a1);
                }
            }
        } else {
            // per spectrum: its own delay, rows before the call from the
            // history, invalid delays and spectra past the launch as zeros
            const uint8_t *hs = hist + int64_t(s) * hist_stride;
#pragma unroll 1
            for (int q = 0; q < 4; ++q) {
                const int m = ltid + NT * q;
                float2 h[T];
                load_tap_pairs<T, n2>(h, taps, m);
#pragma unroll 1
                for (int f = 0; f < PF_S; ++f) {
                    float a0 = 0.f, a1 = 0.f;
                    if (okf[f]) {
                        int64_t i = int64_t(n2) * (F0 + f - T + 1) + 2 * m - cf[f];
#pragma unroll
                        for (int j = 0; j < T; ++j) {
                            a0 = fmaf(float(sample_at(rs, hs, i, H)), h[j].x, a0);
                            a1 = fmaf(float(sample_at(rs, hs, i + 1, H)), h[j].y, a1);
                            i += n2;
                        }
                    }
                    if (MODE == OUT_G) {
                        if (live[f])
                            g_out[(int64_t(s) * M + F0 + f) * N + m] = make_float2(a0, a1);
                    } else {
                        buf[f][lds_pad(m)] = make_float2(a0, a1);
                    }
                }
            }
        }
        if (MODE == OUT_G)
            continue;
        __syncthreads();
        // FFT of spectrum fg by threads tp < n/16, then its channels
        fft_pass0<N>(buf[fg], tp);
        fft_rest<N, 1>(buf[fg], tp, tw_all);
        if (live[fg])
            post_spectrum<N, NTP, MODE>(buf[fg], ph_hi[fg], ph_lo[fg], untangle, gains + int64_t(s) * N,
                                        okf[fg], int64_t(s) * M + F0 + fg, tp, spec8, y_out);
        __syncthreads();                    // the buffers and tables are refilled next step
    }
}

// ---------------------------------------------------------------------------
// Channel counts above what one workgroup's LDS holds (n = 16384, 32768):
// the FFT in two levels (the decomposition behind the paper's Sec. 4 "unzip",
// here with 16 as the first factor).
//
// Level 1 (fft_front_kernel): the first radix-16 Stockham stage, one thread
// per group gam in [0, n/16): inputs z[gam + (n/16) j], outputs
// U[d (n/16) + gam] = exp(-2 pi i gam d / n) DFT16(z[gam + (n/16) j])[d].
// Inputs and outputs of a thread are the same 16 positions, so it runs in
// place on the filtered samples.  Level 2: for each d, Z[d + 16 k'] is the
// (n/16)-point DFT of U[d (n/16) + .] at k'.  Channel k = d + 16 k' pairs
// with n - k in sub-transform (16 - d) mod 16, so fft_post_large_kernel
// transforms the sub-transforms d and 16 - d together (nine rounds per
// spectrum) and finishes both sets of channels.
// ---------------------------------------------------------------------------

template <bool F16>
__global__ __launch_bounds__(256) void fft_front_kernel(float *__restrict__ g, const float2 *__restrict__ twf,
                                                        const float2 *__restrict__ gains, float2 *__restrict__ gpl,
                                                        int n, int M, int mb, int me, int A)
{
    const int gpt = n / 16;                                 // groups per spectrum
    const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
    const int64_t total = int64_t(A) * 2 * (me - mb) * gpt;
    // Side job for the post kernel: this call's per-channel gains of every
    // stream into residue-plane order (position d n/16 + k' holds channel
    // d + 16 k'), so that its lanes read consecutive entries.
    for (int64_t i = e; i < int64_t(A) * 2 * n; i += int64_t(gridDim.x) * 256) {
        const int r = int(i % n);
        gpl[i] = gains[i - r + r / gpt + 16 * (r % gpt)];
    }
    if (e >= total)
        return;
    const int gam = int(e % gpt);
    const int64_t r = e / gpt;                              // (stream, spectrum - mb)
    const int64_t sp = (r / (me - mb)) * M + mb + r % (me - mb);
    // F16: the filtered samples and the stage's outputs as FP16 pairs
    float2 *z = reinterpret_cast<float2 *>(g) + sp * n;
    uint32_t *z16 = reinterpret_cast<uint32_t *>(g) + sp * n;
    float2 v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j)
        v[j] = F16 ? f16_unpair(z16[gam + gpt * j]) : z[gam + gpt * j];
    Dft<16>::run(v);
    const float2 *tw = twf + int64_t(gam) * 16;
#pragma unroll
    for (int d = 0; d < 16; ++d) {
        const float2 y = d == 0 ? v[0] : cmul(v[d], tw[d]);
        if constexpr (F16)
            z16[gam + gpt * d] = f16_pair(y);
        else
            z[gam + gpt * d] = y;
    }
}

// fft_front_kernel's side job alone (calls whose FIR did the first stage):
// the per-channel gains of every stream into residue-plane order.
__global__ __launch_bounds__(256) void gains_planes_kernel(const float2 *__restrict__ gains, float2 *__restrict__ gpl,
                                                           int n, int64_t total)
{
    const int gpt = n / 16;
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i < total) {
        const int r = int(i % n);
        gpl[i] = gains[i - r + r / gpt + 16 * (r % gpt)];
    }
}

template <int NL, int MODE, bool F16 = false>
__global__ __launch_bounds__(NL / 128) void fft_post_large_kernel(
    const float *__restrict__ g, const double *__restrict__ delays,
    const double *__restrict__ phases, const float2 *__restrict__ gains,
    const float2 *__restrict__ tw_sub, const float2 *__restrict__ untangle,
    uint32_t *__restrict__ spec8, float2 *__restrict__ y_out, int *__restrict__ status,
    int M, int D, int mb, int me, int rparts)
{
    constexpr int NS = NL / 16;                             // sub-transform length
    constexpr int NTS = NS / 16;                            // threads per sub-transform
    constexpr int NT = 2 * NTS;
    constexpr int NH = NL / 64;
    __shared__ float2 buf[2][lds_len<NS>()];
    __shared__ float2 ph_hi[NH];
    __shared__ float2 ph_lo[64];

    // block = (work item, part): the nine rounds of a spectrum are split over
    // rparts workgroups, so that a call of few spectra still fills the GPU
    const int lb = xcd_logical(blockIdx.x, gridDim.x);
    const int item = lb / rparts, part = lb % rparts;
    const int rper = (9 + rparts - 1) / rparts;
    const int dd0 = part * rper, dd1 = min(9, dd0 + rper);
    const int p = item & 1;
    const int af = item >> 1;
    const int a = af / (me - mb);
    const int F = mb + af % (me - mb);
    const int tid = threadIdx.x;
    const int half = tid / NTS, tp = tid % NTS;
    const int64_t sp = (int64_t(a) * 2 + p) * M + F;
    const float2 *u = reinterpret_cast<const float2 *>(g) + sp * NL;
    const uint32_t *u16 = reinterpret_cast<const uint32_t *>(g) + sp * NL;   // F16: FP16 pairs
    const float2 *gn = gains + (int64_t(a) * 2 + p) * NL;
    uint16_t *q16 = reinterpret_cast<uint16_t *>(spec8) + sp * NL;

    int c;
    double tau;
    const bool ok = split_delay(delays[sp], D, c, tau);
    if (!ok && tid == 0 && part == 0)
        atomicOr(status, 1);
    phase_tables<NL, NT>(ph_hi, ph_lo, phases[sp], tau, 0.5f, tid);

    for (int dd = dd0; dd < dd1; ++dd) {
        const int dsel = half == 0 ? dd : (16 - dd) & 15;
        float2 *bh = buf[half];
        float2 v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q)
            v[q] = F16 ? f16_unpair(u16[dsel * NS + tp + q * NTS]) : u[dsel * NS + tp + q * NTS];
        Dft<16>::run(v);
#pragma unroll
        for (int r = 0; r < 16; ++r)
            bh[lds_pad(tp * 16 + r)] = v[r];
        __syncthreads();
        fft_rest<NS, 1>(bh, tp, tw_sub);                    // both halves in step (same barriers)

        // channels k = dsel + 16 k' of this half; partner n - k lies in
        // sub-transform (16 - dsel) mod 16, held by the other half (or this
        // one for dsel = 0, 8)
        const bool dup = half == 1 && (dd == 0 || dd == 8);
        if (!dup) {
            // positions kk = 2j, 2j + 1 (j = tp + NTS i) of the plane, four
            // pairs at a time: both tables are in residue-plane order, so a
            // pair's entries are one 16-byte load each and its two int8
            // pairs one 4-byte store (plane dsel, coalesced)
            for (int i0 = 0; i0 < NS / (2 * NTS); i0 += 4) {
                float4 wk[4], gk[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int pos = dsel * NS + 2 * (tp + NTS * (i0 + r));
                    wk[r] = *reinterpret_cast<const float4 *>(untangle + pos);
                    gk[r] = *reinterpret_cast<const float4 *>(gn + pos);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int j = tp + NTS * (i0 + r);
                    float2 Y[2];
#pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        const int kk = 2 * j + e;
                        const int k = dsel + 16 * kk;
                        const int km = (NL - k) & (NL - 1);
                        const int dm = km & 15, km2 = km >> 4;
                        const float2 zk = bh[lds_pad(kk)];
                        const float2 zm = buf[dm == dsel ? half : 1 - half][lds_pad(km2)];
                        const float2 w = e == 0 ? make_float2(wk[r].x, wk[r].y) : make_float2(wk[r].z, wk[r].w);
                        const float2 gg = e == 0 ? make_float2(gk[r].x, gk[r].y) : make_float2(gk[r].z, gk[r].w);
                        const float2 E2 = make_float2(zk.x + zm.x, zk.y - zm.y);
                        const float2 O2 = make_float2(zk.y + zm.y, zm.x - zk.x);
                        const float2 X2 = cadd(E2, cmul(w, O2));
                        const float2 rot = cmul(ph_hi[k >> 6], ph_lo[k & 63]);
                        Y[e] = ok ? cmul(gg, cmul(rot, X2)) : make_float2(0.f, 0.f);
                        if (MODE == OUT_PREQUANT)
                            y_out[sp * NL + k] = Y[e];
                    }
                    if (MODE != OUT_PREQUANT)
                        reinterpret_cast<uint32_t *>(q16)[(dsel * NS) / 2 + j] = quant4(Y[0].x, Y[0].y, Y[1].x, Y[1].y);
                }
            }
        }
        __syncthreads();                                    // the buffers are refilled next round
    }
}

// ---------------------------------------------------------------------------
// Matrix-core (MFMA) variant: the FIR and the radix-16 DFT stages as FP16 or
// BF16 contractions with FP32 accumulation.  Everything else (delay split,
// twiddle and phase generation in FP64 on the host or per spectrum, the
// untangle, phase/gain, quantisation) is the FP32 path's.
//
// FP16 operands hold the 10-bit samples exactly; the taps are scaled by a
// power of two 2^sc (undone on the FP32 result) so that small taps stay out
// of the FP16 subnormal range.  BF16 has 8 significant bits, so operands are
// split as x = hi + lo (both BF16) and a product is formed as
// hi*hi + hi*lo + lo*hi (three MFMAs; the dropped lo*lo term is below 2^-16
// relative).  The filtered samples g travel between the two kernels as FP16
// for FP16 and as FP32 for BF16 (a single BF16 would cost 2^-9).
// ---------------------------------------------------------------------------

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// two floats to an FP16 pair (round to nearest even; one v_cvt_pk_f16_f32)
__device__ __forceinline__ uint32_t pack_f16x2(float lo, float hi)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2{lo, hi}), f16x2));
}

template <int PREC> struct Mx;

template <> struct Mx<FE_PREC_FP16> {
    typedef f16x8 op;
    static constexpr bool split = false;
    __device__ static f32x16 mm32(op a, op b, f32x16 c) { return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0); }
    __device__ static f32x4 mm16(op a, op b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
    __device__ static void put(op &hi, op &lo, int e, float x) { hi[e] = (_Float16)x; (void)lo; }
};

template <> struct Mx<FE_PREC_BF16> {
    typedef bf16x8 op;
    static constexpr bool split = true;
    __device__ static f32x16 mm32(op a, op b, f32x16 c) { return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0); }
    __device__ static f32x4 mm16(op a, op b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
    __device__ static void put(op &hi, op &lo, int e, float x)
    {
        const __bf16 h = (__bf16)x;
        hi[e] = h;
        lo[e] = (__bf16)(x - (float)h);
    }
};

// a*b accumulated into c at the variant's precision (split: hi*hi + hi*lo + lo*hi)
template <int PREC>
__device__ __forceinline__ f32x16 mma32(const typename Mx<PREC>::op &ah, const typename Mx<PREC>::op &al,
                                        const typename Mx<PREC>::op &bh, const typename Mx<PREC>::op &bl,
                                        f32x16 c)
{
    c = Mx<PREC>::mm32(ah, bh, c);
    if constexpr (Mx<PREC>::split) {
        c = Mx<PREC>::mm32(ah, bl, c);
        c = Mx<PREC>::mm32(al, bh, c);
    }
    return c;
}

template <int PREC>
__device__ __forceinline__ f32x4 mma16(const typename Mx<PREC>::op &ah, const typename Mx<PREC>::op &al,
                                       const typename Mx<PREC>::op &bh, const typename Mx<PREC>::op &bl,
                                       f32x4 c)
{
    c = Mx<PREC>::mm16(ah, bh, c);
    if constexpr (Mx<PREC>::split) {
        c = Mx<PREC>::mm16(ah, bl, c);
        c = Mx<PREC>::mm16(al, bh, c);
    }
    return c;
}

// ---------------------------------------------------------------------------
// Kernel 1M: the FIR of Eq. (1) as a banded Toeplitz contraction.
//
// For one column t and a block of 16 consecutive spectra F0' .. F0'+15 that
// share the coarse delay c, with x_q = s[2n(F0' - TK + 1 + q) + t - c]:
//   g[F0'+i][t] = sum_q W_t[i][q] x_q,   W_t[i][q] = h'[t + 2n(q - i)]
// for 0 <= q - i < TK (h' = the taps zero-padded in front to TK), zero
// elsewhere: a 16 x (16 + TK - 1) matrix, half of it zero.  One
// v_mfma_f32_16x16x32 (K-step of 32 rows) takes W_t as A (16 spectra x 32
// rows) and, as B, the 32-row windows of 16 such blocks (the batch): one
// instruction forms 256 outputs of column t.
//
// Workgroup = one stream, 64 columns x 256 spectra (16 blocks); wave w owns
// columns 16w .. 16w+15.  The input rows of the tile are unpacked once into
// LDS as FP16 pairs of rows (the window rows of a column are contiguous), for
// the union of the tile's delays.  Blocks whose spectra do not share one
// delay are formed in several passes, one per delay value, each output
// taking the pass of its own delay.  A tile whose delays spread wider than
// the staging area reads its operands directly from memory instead.
// ---------------------------------------------------------------------------

// two dwords at a 4-byte aligned address (one 8-byte load)
typedef uint32_t u32x2_a4 __attribute__((ext_vector_type(2), aligned(4)));

constexpr int FM_COLS = 64;                // columns per tile
constexpr int FM_SPEC = 256;               // spectra per tile (16 blocks)
constexpr int FM_WMAX = 92;                // staged columns (23 groups of 4): 64 + delay spread + 3

template <int TK> struct FirM {
    static constexpr int KS = (TK + 15 + 31) / 32;         // 32-row K-steps
    static constexpr int ROWS = 16 * 15 + 32 * KS;         // staged rows
    static constexpr int RPW = ROWS / 2 + 1;               // dwords per staged column (odd)
    static constexpr int ZL = 16 + 32 * KS;                // zero-padded tap vector length
};

enum { GOUT_F16 = 0, GOUT_F32 = 1 };

template <int TK, int PREC, int GOUT>
__global__ __launch_bounds__(256, 2) void fir_mfma_kernel(
    const uint8_t *__restrict__ raw, int64_t raw_stride, int64_t Ncall,
    const uint8_t *__restrict__ hist, int64_t hist_stride, int H,
    const float *__restrict__ taps, float tap_scale, float out_scale,
    const double *__restrict__ delays, void *__restrict__ gout,
    int n2, int M, int D, int mb, int me, int ctiles, int ftiles, int chain)
{
    using P = FirM<TK>;
    typedef typename Mx<PREC>::op op;
    constexpr int NPART = Mx<PREC>::split ? 2 : 1;          // tap parts (hi, lo)
    constexpr int PRS = P::ROWS / 2;                         // staged row pairs
    constexpr int IT = (PRS + 7) / 8;                        // row pairs per staging thread
    __shared__ uint32_t stage[FM_WMAX * P::RPW];             // [u][row pair] FP16 x 2
    // tap vectors, 16-bit, [part][col][v]; built first in the staging area
    uint16_t (*zt)[FM_COLS][P::ZL] = reinterpret_cast<uint16_t (*)[FM_COLS][P::ZL]>(stage);
    static_assert(NPART * FM_COLS * P::ZL * 2 <= FM_WMAX * P::RPW * 4, "tap vectors fit the staging area");
    // the same as overlapping pairs: zd[part][col][v] = (z[v], z[v + 1]), so
    // that 8 consecutive taps from any offset are 4 aligned dwords
    __shared__ uint32_t zd[NPART][FM_COLS][P::ZL];
    // delay analysis of two tiles at a time (buffer = tile index parity)
    __shared__ int cdel[2][FM_SPEC];                         // coarse delay, -1 if invalid
    __shared__ uint8_t pass_of[2][FM_SPEC];
    __shared__ int pdel[2][16][16];                          // [block][pass] delay
    __shared__ int wred[2][4][3];                            // per wave: min, max delay, passes

    const int lb = xcd_logical(blockIdx.x, gridDim.x);
    const int ct = lb % ctiles;
    const int rest = lb / ctiles;
    const int nch = (ftiles + chain - 1) / chain;
    const int ch = rest % nch;
    const int s = rest / nch;
    const int t0 = ct * FM_COLS;
    const int fb = ch * chain, fe = min(fb + chain, ftiles);  // this workgroup's spectrum tiles
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint8_t *rs = raw + int64_t(s) * raw_stride;
    const uint8_t *hs = hist + int64_t(s) * hist_stride;
    const double *ds = delays + int64_t(s) * M;

    // ---- tile analysis.  split: one spectrum per thread, wave extremes of the
    // valid delays.  passes (after a barrier): blocks of 16 spectra run one
    // pass per stretch of equal delay; invalid spectra count as the tile's
    // smallest delay (any staged delay: their outputs are zeroed).
    auto load_delay = [&](int f) -> double {
        const int F = mb + f * FM_SPEC + tid;
        return F < me ? ds[F] : 0.0;
    };
    auto split_tile = [&](int f, double d) {
        const int F = mb + f * FM_SPEC + tid;
        int c = -1;
        if (F < me) {
            int cc;
            double tau;
            if (split_delay(d, D, cc, tau))
                c = cc;
        }
        cdel[f & 1][tid] = c;
        int mn = c >= 0 ? c : 0x7fffffff, mx = c;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            mn = min(mn, __shfl_xor(mn, o));
            mx = max(mx, __shfl_xor(mx, o));
        }
        if (lane == 0) {
            wred[f & 1][wave][0] = mn;
            wred[f & 1][wave][1] = mx;
        }
    };
    auto tile_range = [&](int f, int &cmin, int &cmax) {
        const int b = f & 1;
        // (the same in every lane: made scalar so that what depends on it stays scalar)
        cmin = __builtin_amdgcn_readfirstlane(min(min(wred[b][0][0], wred[b][1][0]), min(wred[b][2][0], wred[b][3][0])));
        cmax = __builtin_amdgcn_readfirstlane(max(max(wred[b][0][1], wred[b][1][1]), max(wred[b][2][1], wred[b][3][1])));
        if (cmax < 0)
            cmin = cmax = 0;                                 // no valid spectrum
    };
    auto passes = [&](int f) {
        const int b = f & 1;
        int cmin, cmax;
        tile_range(f, cmin, cmax);
        const int c0 = cdel[b][tid];
        const int ce = c0 >= 0 ? c0 : cmin;
        const int cp = __shfl_up(ce, 1);
        const int j = lane & 15;                             // spectrum within its block
        const bool chg = j != 0 && ce != cp;
        const uint64_t bits = (__builtin_amdgcn_ballot_w64(chg) >> (lane & ~15)) & 0xffffull;
        const int p = __builtin_popcountll(bits & ((2ull << j) - 1));
        pass_of[b][tid] = uint8_t(p);
        const int blk = tid >> 4;
        if (j == 0 || chg)
            pdel[b][blk][p] = ce;
        const int nb = __builtin_popcountll(bits) + 1;
        if (j == 15)
            for (int q = nb; q < 16; ++q)
                pdel[b][blk][q] = ce;                        // fewer passes than the tile's most: repeat the last
        const int mx = max(max(__builtin_amdgcn_readlane(nb, 15), __builtin_amdgcn_readlane(nb, 31)),
                           max(__builtin_amdgcn_readlane(nb, 47), __builtin_amdgcn_readlane(nb, 63)));
        if (lane == 0)
            wred[b][wave][2] = mx;
    };
    // staged columns start on a 4-sample group (5 whole bytes): staged column
    // u holds sample 2n r + 4 gq0 + u of row r, gq0 = floor((t0 - cmax) / 4)
    struct Geo {
        int cmin, cmax, gq0, u0, ngr;
        bool staged;
    };
    auto geometry = [&](int f) {
        Geo G;
        tile_range(f, G.cmin, G.cmax);
        G.gq0 = (t0 - G.cmax) >> 2;                          // arithmetic shift = floor
        G.u0 = (t0 - G.cmax) - 4 * G.gq0;                    // 0 .. 3
        G.ngr = (FM_COLS + G.cmax - G.cmin + G.u0 + 3) >> 2; // groups per staged row
        G.staged = 4 * G.ngr <= FM_WMAX;
        return G;
    };

    // ---- staging of rows [row0, row0 + ROWS) of tile f as FP16 row pairs.
    // Thread (q = tid % 32, prs = tid / 32) takes group q (4 samples in 5
    // bytes) of row pairs prs, prs + 8, ...: each group read as two aligned
    // dwords (in range: every chunk and history row is a multiple of 4
    // bytes).  The loads go to registers first (they are issued a tile ahead,
    // before the previous tile's contraction), the conversion to LDS later.
    const int q = tid & 31, prs = tid >> 5;
    const int gpr = n2 >> 2;                                 // groups per row
    const int hist_g = H >> 2;
    const int ncall_g = int(Ncall >> 2);
    auto group_of = [&](int f, const Geo &G, int pr, int h2) {
        const int row0 = mb + f * FM_SPEC - TK + 1;          // call-relative row of staged row 0
        return gpr * (row0 + 2 * pr + h2) + G.gq0 + q;
    };
    uint32_t dw[IT][2][2];
    const int row_bytes = 5 * gpr;                           // multiple of 4
    // interior tile: every group the staging lanes read lies in the call (the
    // first, group gq0 of row row0, and the last), so the words are read
    // without per-load checks at a scalar row pointer plus one lane offset
    // (the rows of lane pair prs are 2 prs below the pointer; a group's byte
    // phase is the same in every row)
    auto interior = [&](int f, const Geo &G) {
        const int row0 = mb + f * FM_SPEC - TK + 1;
        return G.staged && gpr * row0 + G.gq0 >= 0 && gpr * (row0 + P::ROWS - 1) + G.gq0 + 31 < ncall_g;
    };
    auto stage_load = [&](int f) {
        const Geo G = geometry(f);
        if (interior(f, G)) {
            const int row0 = mb + f * FM_SPEC - TK + 1;
            // gq0 = gpr kr + gr with 0 <= gr < gpr: whole rows kr (negative for
            // coarse delays past the tile's first column) move the scalar row
            // pointer; the lane offset keeps the rest, with one row of margin,
            // so it is never negative (a group's first byte is 5 (gr + q) from
            // its row's start; the dword index is floored)
            const int kr = G.gq0 >= 0 ? G.gq0 / gpr : -((gpr - 1 - G.gq0) / gpr);
            const int gr = G.gq0 - kr * gpr;
            const uint32_t lane_off = uint32_t((2 * prs + 1) * row_bytes + 4 * ((5 * (gr + q)) >> 2));
            gptr8 rp = (gptr8)rs + int64_t(row0 - 1 + kr) * row_bytes;
#pragma unroll
            for (int k = 0; k < IT; ++k) {
#pragma unroll
                for (int h2 = 0; h2 < 2; ++h2) {
                    const u32x2_a4 w = *reinterpret_cast<const u32x2_a4 __attribute__((address_space(1))) *>(rp + lane_off);
                    dw[k][h2][0] = w[0];
                    dw[k][h2][1] = w[1];
                    rp += h2 == 0 ? row_bytes : 15 * row_bytes;   // rows +1, then on to the next 16
                }
            }
            return;
        }
        if (!G.staged || q >= G.ngr)
            return;
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int pr = prs + 8 * k;
#pragma unroll
            for (int h2 = 0; h2 < 2; ++h2) {
                const int ga = group_of(f, G, pr, h2);
                const bool in_hist = ga < 0;
                const bool ok = ga < ncall_g;
                const int byte = 5 * (in_hist ? ga + hist_g : ga);
                const uint8_t *base = in_hist ? hs : rs;
                // unconditional loads (offset 0 stands in for rows outside
                // the call; their words are zeroed at the conversion: a
                // select here would wait for each load in turn)
                const uint32_t *p32 = reinterpret_cast<const uint32_t *>(base) + (ok ? byte >> 2 : 0);
                dw[k][h2][0] = p32[0];
                dw[k][h2][1] = p32[1];
            }
        }
    };
    auto stage_write = [&](int f) {
        const Geo G = geometry(f);
        if (!G.staged || q >= G.ngr)
            return;
        const bool inner = interior(f, G);
        // in an interior tile every group has the byte phase of row 0
        const uint32_t o_in = uint32_t(5 * (G.gq0 + q)) & 3u;
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int pr = prs + 8 * k;
            float x[2][4];
#pragma unroll
            for (int h2 = 0; h2 < 2; ++h2) {
                uint32_t o = o_in, w0 = dw[k][h2][0], w1 = dw[k][h2][1];
                if (!inner) {
                    const int ga = group_of(f, G, pr, h2);
                    o = uint32_t(5 * (ga < 0 ? ga + hist_g : ga)) & 3u;
                    if (ga >= ncall_g)
                        w0 = w1 = 0u;                                // rows past the call
                }
                // big-endian bytes b0..b3 and (b3, b4) of the group
                const uint32_t be0 = __builtin_amdgcn_perm(w1, w0, 0x00010203u + 0x01010101u * o);
                const uint32_t be1 = __builtin_amdgcn_perm(w1, w0, 0x0C0C0000u | ((o + 3u) << 8) | (o + 4u));
                x[h2][0] = float(int32_t(__builtin_amdgcn_sbfe(int32_t(be0), 22u, 10u)));
                x[h2][1] = float(int32_t(__builtin_amdgcn_sbfe(int32_t(be0), 12u, 10u)));
                x[h2][2] = float(int32_t(__builtin_amdgcn_sbfe(int32_t(be0), 2u, 10u)));
                x[h2][3] = float(int32_t(__builtin_amdgcn_sbfe(int32_t(be1), 0u, 10u)));
            }
#pragma unroll
            for (int c4 = 0; c4 < 4; ++c4)
                stage[(4 * q + c4) * P::RPW + pr] = pack_f16x2(x[0][c4], x[1][c4]);
        }
    };

    // ---- contraction of tile f: lane (r16 = lane % 16, kg = lane / 16)
    //   A: W_t[i = r16][32 ks + 8 kg + e];  B: rows 16 b + 32 ks + 8 kg + e of block b = r16;
    //   D: spectra 16 b + 4 kg + e of block b = r16
    const int r16 = lane & 15, kg = lane >> 4;
    const int myb = r16;
    auto contract = [&](int f) {
        const int b = f & 1;
        const Geo G = geometry(f);
        const int npass = __builtin_amdgcn_readfirstlane(max(max(wred[b][0][2], wred[b][1][2]), max(wred[b][2][2], wred[b][3][2])));
        const int F0 = mb + f * FM_SPEC;
        const int64_t row0 = int64_t(F0) - TK + 1;
        int my_pass[4];
#pragma unroll
        for (int e = 0; e < 4; ++e)
            my_pass[e] = pass_of[b][16 * myb + 4 * kg + e];
        // two halves of 8 columns; each half's outputs are stored before the
        // next.  Within a half, CB columns' operands are read together and
        // their MFMAs issued back to back (a pass's delay is the same for
        // every column); CB is what the registers allow beside the next
        // tile's staged words.
        constexpr int CB = P::KS > 1 ? 1 : (Mx<PREC>::split ? 2 : 4);
#pragma unroll 1
        for (int half = 0; half < 2; ++half) {
            f32x4 acc[8];
#pragma unroll
            for (int c4 = 0; c4 < 8; c4 += CB) {
                const int col0 = 16 * wave + 8 * half + c4;
                op ah[CB][P::KS], al[CB][P::KS];
#pragma unroll
                for (int cl = 0; cl < CB; ++cl) {
#pragma unroll
                    for (int ks = 0; ks < P::KS; ++ks) {
                        const int o = 16 + 32 * ks + 8 * kg - r16;
                        const uint32_t *z0 = &zd[0][col0 + cl][o];
                        ah[cl][ks] = __builtin_bit_cast(op, (u32x4{z0[0], z0[2], z0[4], z0[6]}));
                        if constexpr (Mx<PREC>::split) {
                            const uint32_t *z1 = &zd[NPART - 1][col0 + cl][o];
                            al[cl][ks] = __builtin_bit_cast(op, (u32x4{z1[0], z1[2], z1[4], z1[6]}));
                        }
                    }
                    acc[c4 + cl] = f32x4{0.f, 0.f, 0.f, 0.f};
                }
#pragma unroll 1
                for (int ps = 0; ps < npass; ++ps) {
                    const int c = min(max(pdel[b][myb][ps], G.cmin), G.cmax);
                    f32x4 d[CB];
#pragma unroll
                    for (int cl = 0; cl < CB; ++cl)
                        d[cl] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int ks = 0; ks < P::KS; ++ks) {
                        const int rho = 16 * myb + 32 * ks + 8 * kg;
                        op bh[CB], bl[CB];
#pragma unroll
                        for (int cl = 0; cl < CB; ++cl) {
                            const int t = t0 + col0 + cl;
                            if (G.staged) {
                                const int u = col0 + cl + G.cmax - c + G.u0;
                                const uint32_t *sp = stage + u * P::RPW + rho / 2;
                                const u32x4 v4 = {sp[0], sp[1], sp[2], sp[3]};
                                if constexpr (PREC == FE_PREC_FP16) {
                                    bh[cl] = __builtin_bit_cast(op, v4);    // staged FP16 pairs are the operand
                                } else {
#pragma unroll
                                    for (int w = 0; w < 4; ++w) {
                                        // (scalar conversions: a vector FP16x2 -> FP32x2
                                        // conversion miscompiled here)
                                        const float x0 = float(__builtin_bit_cast(_Float16, uint16_t(v4[w])));
                                        const float x1 = float(__builtin_bit_cast(_Float16, uint16_t(v4[w] >> 16)));
                                        Mx<PREC>::put(bh[cl], bl[cl], 2 * w, x0);
                                        Mx<PREC>::put(bh[cl], bl[cl], 2 * w + 1, x1);
                                    }
                                }
                            } else {
#pragma unroll
                                for (int e = 0; e < 8; ++e) {
                                    const int64_t i = int64_t(n2) * (row0 + rho + e) + t - c;
                                    const int x = i < Ncall ? sample_at(rs, hs, i, H) : 0;
                                    Mx<PREC>::put(bh[cl], bl[cl], e, float(x));
                                }
                            }
                        }
#pragma unroll
                        for (int cl = 0; cl < CB; ++cl)
                            d[cl] = mma16<PREC>(ah[cl][ks], al[cl][ks], bh[cl], bl[cl], d[cl]);
                    }
#pragma unroll
                    for (int cl = 0; cl < CB; ++cl)
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (my_pass[e] == ps)
                                acc[c4 + cl][e] = d[cl][e];
                }
            }

            // outputs: lane holds spectra 16 b + 4 kg + e at 8 consecutive columns
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int fl = 16 * myb + 4 * kg + e;
                const int F = F0 + fl;
                if (F >= me)
                    continue;
                const bool ok = cdel[b][fl] >= 0;
                const int64_t base = (int64_t(s) * M + F) * n2 + t0 + 16 * wave + 8 * half;
                if constexpr (GOUT == GOUT_F16) {
                    uint32_t w[4];
#pragma unroll
                    for (int qq = 0; qq < 4; ++qq) {
                        const float v0 = ok ? acc[2 * qq][e] * out_scale : 0.f;
                        const float v1 = ok ? acc[2 * qq + 1][e] * out_scale : 0.f;
                        w[qq] = pack_f16x2(v0, v1);
                    }
                    *reinterpret_cast<u32x4 *>(static_cast<_Float16 *>(gout) + base) = u32x4{w[0], w[1], w[2], w[3]};
                } else {
                    // FP32 store; for FP16 streams the value is the FP16-rounded one
                    f32x4 *dst = reinterpret_cast<f32x4 *>(static_cast<float *>(gout) + base);
#pragma unroll
                    for (int qq = 0; qq < 2; ++qq) {
                        f32x4 v;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            float x = ok ? acc[4 * qq + r][e] * out_scale : 0.f;
                            if constexpr (PREC == FE_PREC_FP16)
                                x = float((_Float16)x);
                            v[r] = x;
                        }
                        dst[qq] = v;
                    }
                }
            }
        }
    };

    // ---- tap vectors (once): zt[col][16 + j] = h'[t + 2n j] (scaled), zero
    // elsewhere; lanes take consecutive columns (coalesced), all loads first
    {
        const int col = tid & 63, j0 = tid >> 6;
        constexpr int JPT = (TK + 3) / 4;
        float hv[JPT];
#pragma unroll
        for (int qq = 0; qq < JPT; ++qq) {
            const int j = j0 + 4 * qq;
            hv[qq] = j < TK ? taps[(t0 + col) + int64_t(n2) * j] * tap_scale : 0.f;
        }
        for (int v = j0; v < P::ZL; v += 4)
            if (v < 16 || v >= 16 + TK)
                for (int part = 0; part < NPART; ++part)
                    zt[part][col][v] = 0;
#pragma unroll
        for (int qq = 0; qq < JPT; ++qq) {
            const int j = j0 + 4 * qq;
            if (j < TK) {
                const float hh = hv[qq];
                if constexpr (Mx<PREC>::split) {
                    const __bf16 h1 = (__bf16)hh;
                    const __bf16 h2 = (__bf16)(hh - (float)h1);
                    zt[0][col][16 + j] = __builtin_bit_cast(uint16_t, h1);
                    zt[1][col][16 + j] = __builtin_bit_cast(uint16_t, h2);
                } else {
                    zt[0][col][16 + j] = __builtin_bit_cast(uint16_t, (_Float16)hh);
                }
            }
        }
    }
    // ---- the first two tiles' delays
    split_tile(fb, load_delay(fb));
    if (fb + 1 < fe)
        split_tile(fb + 1, load_delay(fb + 1));
    __syncthreads();
    for (int e = tid; e < NPART * FM_COLS * P::ZL; e += 256) {
        const int part = e / (FM_COLS * P::ZL);
        const int col = (e / P::ZL) % FM_COLS, v = e % P::ZL;
        const uint32_t lo = zt[part][col][v];
        const uint32_t hi = v + 1 < P::ZL ? zt[part][col][v + 1] : 0u;
        zd[part][col][v] = lo | (hi << 16);
    }
    passes(fb);
    if (fb + 1 < fe)
        passes(fb + 1);
    __syncthreads();                                         // zd and the pass tables are out; zt is free
    stage_load(fb);
    stage_write(fb);
    double d2 = fb + 2 < fe ? load_delay(fb + 2) : 0.0;
    __syncthreads();

    // ---- the chain: tile f+1's rows and tile f+3's delays are loaded while
    // tile f is contracted; tile f+2 is analysed behind it
    for (int f = fb; f < fe; ++f) {
        if (f + 1 < fe)
            stage_load(f + 1);
        const double d3 = f + 3 < fe ? load_delay(f + 3) : 0.0;
        contract(f);
        __syncthreads();                                     // the staging area and tile f's tables are free
        if (f + 1 < fe)
            stage_write(f + 1);
        if (f + 2 < fe)
            split_tile(f + 2, d2);
        d2 = d3;
        __syncthreads();
        if (f + 2 < fe)
            passes(f + 2);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Kernel 2M: FFT + post-processing with the radix-16 stages on the matrix
// cores.
//
// Stockham formulation over the n complex points z (z[m] = g[2m] + i g[2m+1]).
// Stage s (R_s = n / 16^s points per sub-transform, R' = R_s / 16) takes
// group gam in [0, n/16), reads its 16 inputs at
//   in(gam, j) = (gam mod R') + R' (j + 16 (gam div R')),      j = 0..15,
// forms the 16-point DFT, multiplies output d by exp(-2 pi i (gam mod R') d / R_s)
// and writes it to out(gam, d) = gam + (n/16) d.  After the last stage the
// points are in natural order.  As a matrix product: 32 groups at a time
// (the MFMA's N), the 16 complex inputs interleaved (re, im) as K = 32, the
// outputs as M = 32 rows (16 real parts, then 16 imaginary parts), so A is
// the real 32 x 32 form of the DFT-16 matrix, scaled by 1/4 so that values
// cannot grow out of FP16 range (the 4^stages is returned with the phase
// table).  v_mfma_f32_32x32x16 takes K in two halves.  A leftover radix
// (2, 4 or 8, when n is not a power of 16) runs in FP32 on the vector ALUs,
// except for FP16 at n = 8192 = 16^2 x 32, whose last stage is radix 32 on
// the matrix cores: the real 64 x 64 form of the DFT-32 matrix (unscaled:
// its outputs stay in FP32) as two 32-row tiles, K in four steps, 32 groups
// (R' = 1, no twiddles) per column block.  It costs four times the matrix
// work of a radix-16 stage, so it only matches radix 16 + the radix-2 pass
// there (FFT/post 0.213 ms either way on 4 antennas x 2^24 samples) and
// loses for BF16 (hi + lo: 0.287 against 0.282) and at n = 512 (FP16 0.045
// against 0.042, BF16 0.075 against 0.055), which keep the radix-2 pass.
// ---------------------------------------------------------------------------

template <int N, int PREC> struct MPlan {
    static constexpr bool R32 = PREC == FE_PREC_FP16 && N == 8192;   // last stage radix 32 (matrix cores)
    static constexpr int S16 = N >= 4096 ? (R32 ? 2 : 3) : 2;       // radix-16 matrix stages
    static constexpr int RL = R32 ? 1 : N >> (4 * S16);     // leftover radix: 1, 2, 4, 8
    static constexpr int G = N / 16;                        // groups per matrix stage
    static constexpr int NT = N / 16 >= 64 ? N / 16 : 64;   // threads
    static constexpr int NW = NT / 64;
    static constexpr int CB = (G + 31) / 32;                // 32-group column blocks
    static constexpr int CPW = (CB + NW - 1) / NW;          // column blocks per wave
};

// R' of matrix stage s
template <int N> __host__ __device__ constexpr int mstage_rn(int s)
{
    int r = N;
    for (int i = 0; i <= s; ++i)
        r /= 16;
    return r;
}

// One matrix stage reading its inputs from LDS (stages >= 1) or from the
// registers already loaded (stage 0), writing outputs back to LDS.
template <int N, int PREC, int S>
__device__ __forceinline__ void mfma_stage(float2 *__restrict__ buf, typename Mx<PREC>::op (&Bh)[MPlan<N, PREC>::CPW][2],
                                           typename Mx<PREC>::op (&Bl)[MPlan<N, PREC>::CPW][2],
                                           const typename Mx<PREC>::op (&Ah)[2],
                                           const typename Mx<PREC>::op (&Al)[2],
                                           const float2 *__restrict__ tw16, int wave, int lane)
{
    using P = MPlan<N, PREC>;
    constexpr int RN = mstage_rn<N>(S);
    constexpr bool TWID = RN > 1;
    // FP16: stages hand their outputs to the next matrix stage as FP16 pairs
    // (exactly the next B operand); the last matrix stage writes FP32
    constexpr bool IN16 = PREC == FE_PREC_FP16 && S > 0;
    constexpr bool OUT16 = PREC == FE_PREC_FP16 && (S + 1 < P::S16 || P::R32);
    uint32_t *buf32 = reinterpret_cast<uint32_t *>(buf);
    const int n32 = lane & 31, h = lane >> 5;
    if constexpr (S > 0) {
#pragma unroll
        for (int u = 0; u < P::CPW; ++u) {
            const int gam = 32 * (wave * P::CPW + u) + n32;
            const bool valid = P::G % 32 == 0 || gam < P::G;   // only n = 256 has idle lanes
            // in(gam, j) = base + RN j.  Padded, the j term is a constant offset
            // when RN >= 16 (RN j is a multiple of 16) or RN = 1 (16 gam + j
            // stays within one padded row); RN = 2, 4, 8 pads each index.
            const int base = (gam % RN) + RN * 16 * (gam / RN) + RN * 4 * h;
            constexpr bool LIN = RN >= 16 || RN == 1;
            const int pb = lds_pad(base);
            constexpr int STEP = RN >= 16 ? RN + RN / 16 : 1;
            auto at = [&](int m) { return LIN ? pb + STEP * m : lds_pad(base + RN * m); };
#pragma unroll
            for (int kap = 0; kap < 2; ++kap) {
                if constexpr (IN16) {
                    u32x4 w;
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        w[e] = valid ? buf32[at(8 * kap + e)] : 0u;
                    Bh[u][kap] = __builtin_bit_cast(typename Mx<PREC>::op, w);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const float2 v = valid ? buf[at(8 * kap + e)] : make_float2(0.f, 0.f);
                        Mx<PREC>::put(Bh[u][kap], Bl[u][kap], 2 * e, v.x);
                        Mx<PREC>::put(Bh[u][kap], Bl[u][kap], 2 * e + 1, v.y);
                    }
                }
            }
        }
    }
    f32x16 acc[P::CPW];
#pragma unroll
    for (int u = 0; u < P::CPW; ++u) {
        acc[u] = f32x16{};
#pragma unroll
        for (int kap = 0; kap < 2; ++kap)
            acc[u] = mma32<PREC>(Ah[kap], Al[kap], Bh[u][kap], Bl[u][kap], acc[u]);
    }
    if constexpr (S > 0)
        __syncthreads();                                    // every input read before any output lands
#pragma unroll
    for (int u = 0; u < P::CPW; ++u) {
        const int gam = 32 * (wave * P::CPW + u) + n32;
        if (P::G % 32 != 0 && gam >= P::G)
            continue;
        // lane holds outputs d = 8 (t / 4) + 4 h + t % 4: re in acc[t], im in acc[t + 8]
        // twiddles w^d, w = exp(-2 pi i (gam mod R') / 16 R') for this lane's
        // d = 4h .. 4h+3 and 8+4h .. 11+4h: one load of the table's pair
        // (w^4h, w^4h+1); w is the second times the conjugate of the first,
        // w^4 comes from the partner lane (lane ^ 32, same group, other h)
        // through the LDS crossbar, and the rest follow by products (at most
        // five deep: rounding near 3e-7, far below the operands' precision)
        float2 tw[8];
        if constexpr (TWID) {
            const float4 *tp = reinterpret_cast<const float4 *>(tw16 + (int64_t(S) * P::G + gam) * 16);
            const float4 w0 = tp[2 * h];
            const float2 a = make_float2(w0.x, w0.y), b = make_float2(w0.z, w0.w);
            const float2 w = make_float2(b.x * a.x + b.y * a.y, b.y * a.x - b.x * a.y);     // b conj(a)
            const float2 pa = make_float2(__shfl_xor(a.x, 32), __shfl_xor(a.y, 32));
            const float2 w4 = h ? a : pa;
            const float2 w8 = cmul(w4, w4);
            tw[0] = a;
            tw[1] = b;
            tw[2] = cmul(b, w);
            tw[3] = cmul(tw[2], w);
            tw[4] = cmul(a, w8);
            tw[5] = cmul(b, w8);
            tw[6] = cmul(tw[5], w);
            tw[7] = cmul(tw[6], w);
        }
        // out(gam, d) = gam + G d, G a multiple of 16 (or the whole array when G = 16)
        const int pw = lds_pad(gam + P::G * 4 * h);
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int dd = 8 * (t / 4) + t % 4;                 // d - 4 h
            float2 y = make_float2(acc[u][t], acc[u][t + 8]);
            if constexpr (TWID)
                y = cmul(y, tw[t]);
            if constexpr (OUT16)
                buf32[pw + (P::G + P::G / 16) * dd] = pack_f16x2(y.x, y.y);
            else
                buf[pw + (P::G + P::G / 16) * dd] = y;
        }
    }
    __syncthreads();
}

// The radix-32 last stage (MPlan<N, PREC>::R32): group gam in [0, n/32) reads its
// 32 inputs at in(gam, j) = 32 gam + j (FP16 pairs, or float32 split hi + lo
// for BF16) and writes its DFT-32 output d to gam + (n/32) d; no twiddles.
// A32h/A32l hold this lane's A operands [row tile][K step] of the real
// 64 x 64 DFT-32 matrix.
template <int N, int PREC>
__device__ __forceinline__ void mfma_stage32(float2 *__restrict__ buf, const typename Mx<PREC>::op (&A32h)[2][4],
                                             const typename Mx<PREC>::op (&A32l)[2][4], int wave, int lane)
{
    using P = MPlan<N, PREC>;
    typedef typename Mx<PREC>::op op;
    constexpr int G32 = N / 32;                             // groups
    constexpr int CB32 = (G32 + 31) / 32;                   // 32-group column blocks
    constexpr int CPW32 = (CB32 + P::NW - 1) / P::NW;       // column blocks per wave
    constexpr bool IN16 = PREC == FE_PREC_FP16;             // the radix-16 stage before wrote FP16 pairs
    uint32_t *buf32 = reinterpret_cast<uint32_t *>(buf);
    const int n32 = lane & 31, h = lane >> 5;
    op Bh[CPW32][4], Bl[CPW32][4];
#pragma unroll
    for (int u = 0; u < CPW32; ++u) {
        const int cb = wave * CPW32 + u;
        const int gam = 32 * cb + n32;
        const bool valid = cb < CB32 && gam < G32;
        // K step kap takes inputs j = 8 kap + 4 h + e (e < 4), interleaved (re, im)
        const int base = 32 * gam + 4 * h;
#pragma unroll
        for (int kap = 0; kap < 4; ++kap) {
            if constexpr (IN16) {
                u32x4 w;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    w[e] = valid ? buf32[lds_pad(base + 8 * kap + e)] : 0u;
                Bh[u][kap] = __builtin_bit_cast(op, w);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float2 v = valid ? buf[lds_pad(base + 8 * kap + e)] : make_float2(0.f, 0.f);
                    Mx<PREC>::put(Bh[u][kap], Bl[u][kap], 2 * e, v.x);
                    Mx<PREC>::put(Bh[u][kap], Bl[u][kap], 2 * e + 1, v.y);
                }
            }
        }
    }
    f32x16 acc[CPW32][2];
#pragma unroll
    for (int u = 0; u < CPW32; ++u)
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            acc[u][mt] = f32x16{};
#pragma unroll
            for (int kap = 0; kap < 4; ++kap)
                acc[u][mt] = mma32<PREC>(A32h[mt][kap], A32l[mt][kap], Bh[u][kap], Bl[u][kap], acc[u][mt]);
        }
    __syncthreads();                                        // every input read before any output lands
#pragma unroll
    for (int u = 0; u < CPW32; ++u) {
        const int cb = wave * CPW32 + u;
        const int gam = 32 * cb + n32;
        if (cb >= CB32 || gam >= G32)
            continue;
        // lane holds rows m = 8 (v / 4) + 4 h + v % 4 of both tiles: output d = m,
        // real part in tile 0, imaginary part in tile 1
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int d = 8 * (v / 4) + 4 * h + v % 4;
            buf[lds_pad(gam + G32 * d)] = make_float2(acc[u][0][v], acc[u][1][v]);
        }
    }
    __syncthreads();
}

template <int N, int PREC, int S>
__device__ __forceinline__ void mfma_stages(float2 *buf, typename Mx<PREC>::op (&Bh)[MPlan<N, PREC>::CPW][2],
                                            typename Mx<PREC>::op (&Bl)[MPlan<N, PREC>::CPW][2],
                                            const typename Mx<PREC>::op (&Ah)[2],
                                            const typename Mx<PREC>::op (&Al)[2],
                                            const float2 *tw16, int wave, int lane)
{
    if constexpr (S < MPlan<N, PREC>::S16) {
        mfma_stage<N, PREC, S>(buf, Bh, Bl, Ah, Al, tw16, wave, lane);
        mfma_stages<N, PREC, S + 1>(buf, Bh, Bl, Ah, Al, tw16, wave, lane);
    }
}

// The body of kernel 2M for stream spectrum sp = (2 a + p) M + F by threads
// tid < MPlan<N, PREC>::NT, with LDS buf (lds_len<N>), ph_hi (max(N/64, 1)) and
// ph_lo (64).  sync: a workgroup barrier after the stage-0 operand loads,
// before the first LDS write (for a workgroup that transformed another
// spectrum before).  MODE OUT_REG leaves the int8 dwords in qreg.
template <int N, int PREC, int MODE>
__device__ __forceinline__ void fft_mfma_block(
    int a, int p, int64_t sp, int tid, bool sync, float2 *__restrict__ buf, float2 *__restrict__ ph_hi,
    float2 *__restrict__ ph_lo, const void *__restrict__ g, const double *__restrict__ delays,
    const double *__restrict__ phases, const float2 *__restrict__ gains,
    const float2 *__restrict__ tw16, const float2 *__restrict__ untangle,
    const u32x4 *__restrict__ dft_a, uint32_t *__restrict__ spec8, float2 *__restrict__ y_out,
    int *__restrict__ status, int D, uint32_t *qreg = nullptr)
{
    using P = MPlan<N, PREC>;
    typedef typename Mx<PREC>::op op;
    constexpr int NT = P::NT;
    const int lane = tid & 63, wave = tid >> 6;
    const int n32 = lane & 31, h = lane >> 5;

    // stage-0 operands straight from g: in(gam, j) = gam + (n/16) j (loaded
    // non-temporally, like the FP32 kernel: g is read once, and the int8
    // spectra written here should stay cached for the corner turn)
    op Bh[P::CPW][2], Bl[P::CPW][2];
#pragma unroll
    for (int u = 0; u < P::CPW; ++u) {
        const int gam = 32 * (wave * P::CPW + u) + n32;
        const bool valid = P::G % 32 == 0 || gam < P::G;   // only n = 256 has idle lanes
#pragma unroll
        for (int kap = 0; kap < 2; ++kap) {
            if constexpr (PREC == FE_PREC_FP16) {
                // the stored FP16 pairs are the operand
                u32x4 w;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int j = 8 * kap + 4 * h + e;
                    w[e] = valid ? __builtin_nontemporal_load(static_cast<const uint32_t *>(g) + sp * N + gam + P::G * j)
                                 : 0u;
                }
                Bh[u][kap] = __builtin_bit_cast(op, w);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int j = 8 * kap + 4 * h + e;
                    const float2 v = valid ? load_nt(static_cast<const float2 *>(g) + sp * N + gam + P::G * j)
                                           : make_float2(0.f, 0.f);
                    Mx<PREC>::put(Bh[u][kap], Bl[u][kap], 2 * e, v.x);
                    Mx<PREC>::put(Bh[u][kap], Bl[u][kap], 2 * e + 1, v.y);
                }
            }
        }
    }
    // the real 32 x 32 DFT-16 matrix (scaled 1/4) as this lane's A operands
    op Ah[2], Al[2];
#pragma unroll
    for (int kap = 0; kap < 2; ++kap) {
        const u32x4 vh = dft_a[(kap * 2 + 0) * 64 + lane];
        Ah[kap] = __builtin_bit_cast(op, vh);
        if constexpr (Mx<PREC>::split) {
            const u32x4 vl = dft_a[(kap * 2 + 1) * 64 + lane];
            Al[kap] = __builtin_bit_cast(op, vl);
        }
    }

    int c;
    double tau;
    const bool ok = split_delay(delays[sp], D, c, tau);
    if (!ok && tid == 0)
        atomicOr(status, 1);
    if (sync)
        __syncthreads();                                    // the previous spectrum's readers are done with LDS
    constexpr float unscale = float(1 << (2 * P::S16));    // 4^stages
    phase_tables<N, NT>(ph_hi, ph_lo, phases[sp], tau, 0.5f * unscale, tid);

    mfma_stages<N, PREC, 0>(buf, Bh, Bl, Ah, Al, tw16, wave, lane);

    if constexpr (P::R32) {
        // the DFT-32 operands follow the DFT-16 ones in the table
        op A32h[2][4], A32l[2][4];
        const u32x4 *a32 = dft_a + 2 * 2 * 64;
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int kap = 0; kap < 4; ++kap) {
                A32h[mt][kap] = __builtin_bit_cast(op, a32[((mt * 4 + kap) * 2 + 0) * 64 + lane]);
                if constexpr (Mx<PREC>::split)
                    A32l[mt][kap] = __builtin_bit_cast(op, a32[((mt * 4 + kap) * 2 + 1) * 64 + lane]);
                else
                    A32l[mt][kap] = A32h[mt][kap];              // unused (no lo operand)
            }
        mfma_stage32<N, PREC>(buf, A32h, A32l, wave, lane);
    }
    if constexpr (P::RL > 1) {
        // leftover radix RL in FP32: group gam reads RL gam + j, writes gam + (n/RL) d
        constexpr int GR = N / P::RL;
        constexpr int PER = GR / NT;
        float2 v[PER][P::RL];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int gam = tid + NT * q;
#pragma unroll
            for (int j = 0; j < P::RL; ++j)
                v[q][j] = buf[lds_pad(P::RL * gam + j)];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int gam = tid + NT * q;
            Dft<P::RL>::run(v[q]);
#pragma unroll
            for (int d = 0; d < P::RL; ++d)
                buf[lds_pad(gam + GR * d)] = v[q][d];
        }
        __syncthreads();
    }

    post_spectrum<N, NT, MODE, true>(buf, ph_hi, ph_lo, untangle, gains + (int64_t(a) * 2 + p) * N, ok, sp,
                                     tid, spec8, y_out, true, qreg);
}

template <int N, int PREC, int MODE>
__global__ __launch_bounds__((MPlan<N, PREC>::NT), (N >= 8192 ? 2 : 4)) void fft_mfma_kernel(
    const void *__restrict__ g, const double *__restrict__ delays,
    const double *__restrict__ phases, const float2 *__restrict__ gains,
    const float2 *__restrict__ tw16, const float2 *__restrict__ untangle,
    const u32x4 *__restrict__ dft_a, uint32_t *__restrict__ spec8, float2 *__restrict__ y_out,
    int *__restrict__ status, int M, int D, int mb, int me)
{
    constexpr int NH = N / 64;
    __shared__ float2 buf[lds_len<N>()];
    __shared__ float2 ph_hi[NH < 1 ? 1 : NH];
    __shared__ float2 ph_lo[64];
    const int item = xcd_logical(blockIdx.x, gridDim.x);
    const int p = item & 1;
    const int af = item >> 1;
    const int a = af / (me - mb);
    const int F = mb + af % (me - mb);
    const int64_t sp = (int64_t(a) * 2 + p) * M + F;
    fft_mfma_block<N, PREC, MODE>(a, p, sp, threadIdx.x, false, buf, ph_hi, ph_lo, g, delays, phases, gains,
                                  tw16, untangle, dft_a, spec8, y_out, status, D);
}

// Kernel 2MH: kernel 2M with the corner turn folded in (FP16/BF16, int8
// output), organised as kernel 2H: one workgroup per (antenna, run of SPW
// consecutive spectra) transforms and finishes both polarizations of each
// spectrum in turn, keeping the int8 dwords in registers, and writes every
// channel's 4 SPW bytes straight into the heap.
template <int N, int PREC, int SPW>
__global__ __launch_bounds__((MPlan<N, PREC>::NT), (N >= 8192 ? 2 : 4)) void fft_mfma_heap_kernel(
    const void *__restrict__ g, const double *__restrict__ delays,
    const double *__restrict__ phases, const float2 *__restrict__ gains,
    const float2 *__restrict__ tw16, const float2 *__restrict__ untangle,
    const u32x4 *__restrict__ dft_a, int8_t *__restrict__ out, int *__restrict__ status, int M, int D, int S)
{
    constexpr int NT = MPlan<N, PREC>::NT;
    constexpr int NH = N / 64;
    constexpr int P = N / 2 / NT;          // channel pairs per thread
    constexpr int Q = 2 * SPW;
    __shared__ float2 buf[lds_len<N>()];
    __shared__ float2 ph_hi[NH < 1 ? 1 : NH];
    __shared__ float2 ph_lo[64];
    const int runs = M / SPW;
    const int item = xcd_logical(blockIdx.x, gridDim.x);
    const int a = item / runs;
    const int F0 = (item % runs) * SPW;

    uint32_t q[Q][P];
#pragma unroll
    for (int u = 0; u < Q; ++u)
#pragma unroll
        for (int i = 0; i < P; ++i)
            q[u][i] = 0u;
#pragma unroll 1
    for (int fp = 0; fp < Q; ++fp) {
        const int f = fp >> 1, p = fp & 1;
        // fresh copies of the thread index and table bases per pass, so that
        // the loads derived from them are not hoisted out of the loop
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const float2 *tw = tw16, *ut = untangle;
        const u32x4 *da = dft_a;
        asm volatile("" : "+s"(tw), "+s"(ut), "+s"(da));
        const int64_t sp = (int64_t(a) * 2 + p) * M + F0 + f;
        uint32_t qn[P];
        fft_mfma_block<N, PREC, OUT_REG>(a, p, sp, tid, fp > 0, buf, ph_hi, ph_lo, g, delays, phases, gains,
                                         tw, ut, da, nullptr, nullptr, status, D, qn);
#pragma unroll
        for (int i = 0; i < P; ++i) {
#pragma unroll
            for (int u = 0; u + 1 < Q; ++u)
                q[u][i] = q[u + 1][i];
            q[Q - 1][i] = qn[i];
        }
    }
    heap_store<N, NT, SPW, P>(q, out, a, M, S, F0, int(threadIdx.x));
}

// ---------------------------------------------------------------------------
// Kernel 3: corner turn of the int8 spectra into heaps,
//   [A][2][M][n][2]  ->  [A][M/S][n][S][2][2].
// A workgroup moves a tile of 64 spectra x 64 channels of one antenna through
// LDS: it reads 128-byte rows (one pol, one spectrum, 64 channels) and writes
// runs of consecutive spectra of one channel (contiguous within a heap).
// Both sides are non-temporal: the spectra are dead after this read and the
// heaps are not read again on the device, so neither displaces the next
// call's input from the last-level cache nor is left there dirty.
// ---------------------------------------------------------------------------

constexpr int CT = 64;                     // tile edge (spectra and channels)

// spec8 holds each spectrum either in channel order or, for the two-level
// FFT (ns = n/16), as 16 planes of ns channels: position j = d ns + k' is
// channel d + 16 k'.  A tile never straddles planes (ns is a multiple of 64).
// The body for block b of a launch over spectrum tiles ft0 .. ft0 + ftiles - 1
// (all antennas); t16 is an LDS tile.
__device__ __forceinline__ void corner_turn_block(
    int b, int ft0, uint16_t (*__restrict__ t16)[2 * CT + 2],
    const uint32_t *__restrict__ spec8, int8_t *__restrict__ out, int M, int n, int S,
    int ftiles, int ktiles, int ns)
{
    // t16[f][2k + p] = (re, im) of channel k0+k, pol p, spectrum F0+f
    const int kt = b % ktiles;
    const int rest = b / ktiles;
    const int ft = ft0 + rest % ftiles;
    const int a = rest / ftiles;
    const int F0 = ft * CT, k0 = kt * CT;
    const int tid = threadIdx.x;

    // read: row r = (f, p) holds 32 dwords (64 channels); lanes take a dword each
    const int kk = (tid & 31) * 2;
    for (int r = tid >> 5; r < 2 * CT; r += 256 / 32) {
        const int f = r >> 1, p = r & 1;
        const int F = F0 + f;
        uint32_t w = 0;
        if (F < M)
            w = __builtin_nontemporal_load(spec8 + ((int64_t(a) * 2 + p) * M + F) * (n / 2) + (k0 + kk) / 2);
        t16[f][2 * kk + p] = uint16_t(w);
        t16[f][2 * (kk + 1) + p] = uint16_t(w >> 16);
    }
    __syncthreads();

    // write: lane = spectrum, so a wave stores 64 consecutive dwords of a channel
    const int f = tid & (CT - 1);
    const int F = F0 + f;
    // channel of tile position k: c0 + cs k
    const int c0 = ns ? k0 / ns + 16 * (k0 % ns) : k0;
    const int cs = ns ? 16 : 1;
    if (F < M) {
        for (int k = tid >> 6; k < CT; k += 256 / CT) {
            const uint32_t d = *reinterpret_cast<const uint32_t *>(&t16[f][2 * k]);
            const int64_t idx = ((int64_t(a) * (M / S) + F / S) * n + c0 + cs * k) * S + (F % S);
            __builtin_nontemporal_store(d, reinterpret_cast<uint32_t *>(out) + idx);
        }
    }
}

__global__ __launch_bounds__(256) void corner_turn_kernel(
    const uint32_t *__restrict__ spec8, int8_t *__restrict__ out, int M, int n, int S,
    int ftiles, int ktiles, int ns)
{
    __shared__ uint16_t t16[CT][2 * CT + 2];
    corner_turn_block(blockIdx.x, 0, t16, spec8, out, M, n, S, ftiles, ktiles, ns);
}

// ---------------------------------------------------------------------------
// Batches: kernels driven by job lists spanning the member streams, so that
// a batch step runs one FIR launch per tap count, one FFT/post launch per
// channel count and one corner-turn launch for all its FP32 members.  Job j
// owns blocks [begin_j, begin_{j+1}) (the list is in block order); a block
// finds its job by a scan of the (at most a few dozen) entries, which every
// lane reads alike.
// ---------------------------------------------------------------------------

struct FirJob {
    const uint8_t *raw;
    int64_t raw_stride;
    const uint8_t *hist;
    int64_t hist_stride;
    const float *taps;
    const double *delays;
    float *g;
    int H, n2, M, D, R, colblocks, runs, mb, me, moff, mrows, begin;
};

struct PostJob {
    const float *g;
    const double *delays;
    const double *phases;
    const float2 *gains;
    const float2 *tw;
    const float2 *untangle;
    uint32_t *spec8;
    int *status;
    int M, D, begin, pad;
};

struct TurnJob {
    const uint32_t *spec8;
    int8_t *out;
    int M, n, S, ftiles, ktiles, ns, begin, pad;
};

// per stream s < streams: dst[s dst_stride + i], i < len (32-bit words) =
// 0 for i < z, src1[s src1_stride + i - z] for i < z + h, else
// src2[s src2_stride + src2_off + i - z - h]; the job owns words
// [begin, begin + streams len) of the launch
struct CopyJob {
    uint32_t *dst;
    const uint32_t *src1;
    const uint32_t *src2;
    int64_t dst_stride, src1_stride, src2_stride, src2_off, z, h, len, begin;
    int streams, pad;
};

template <typename J>
__device__ __forceinline__ int find_job(const J *__restrict__ jobs, int njobs, int64_t b)
{
    int j = 0;
    while (j + 1 < njobs && jobs[j + 1].begin <= b)
        ++j;
    return j;
}

template <int T>
__global__ __launch_bounds__(FIR_THREADS, FIR_WG_PER_CU(T)) void fir_jobs_kernel(const FirJob *__restrict__ jobs,
                                                                                  int njobs)
{
    __shared__ int s_c[FIR_SEG];
    const int b = blockIdx.x;
    const FirJob &J = jobs[find_job(jobs, njobs, b)];
    fir_block<T>(b - J.begin, s_c, J.raw, J.raw_stride, J.hist, J.hist_stride, J.H, J.taps, J.delays, J.g, J.n2,
                 J.M, J.D, J.R, J.colblocks, J.runs, J.mb, J.me, J.moff, J.mrows);
}

template <int N>
__global__ __launch_bounds__(N / 16, (N / 16 >= 256 ? 4 : 1)) void post_jobs_kernel(const PostJob *__restrict__ jobs,
                                                                                    int njobs)
{
    constexpr int NH = N / 64;
    __shared__ float2 buf[lds_len<N>()];
    __shared__ float2 ph_hi[NH < 1 ? 1 : NH];
    __shared__ float2 ph_lo[64];
    __shared__ float2 tws[TW_PASS1];
    const int b = blockIdx.x;
    const PostJob &J = jobs[find_job(jobs, njobs, b)];
    fft_post_block<N, OUT_INT8>(b - J.begin, true, threadIdx.x, buf, ph_hi, ph_lo, tws, J.g, J.delays, J.phases,
                                J.gains, J.tw, J.untangle, J.spec8, nullptr, J.status, J.M, J.D, 0, J.M);
}

__global__ __launch_bounds__(256) void turn_jobs_kernel(const TurnJob *__restrict__ jobs, int njobs)
{
    __shared__ uint16_t t16[CT][2 * CT + 2];
    const int b = blockIdx.x;
    const TurnJob &J = jobs[find_job(jobs, njobs, b)];
    corner_turn_block(b - J.begin, 0, t16, J.spec8, J.out, J.M, J.n, J.S, J.ftiles, J.ktiles, J.ns);
}

__global__ void copy_jobs_kernel(const CopyJob *__restrict__ jobs, int njobs, int64_t total)
{
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
         e += int64_t(gridDim.x) * blockDim.x) {
        const CopyJob &J = jobs[find_job(jobs, njobs, e)];
        const int64_t w = e - J.begin, s = w / J.len, i = w % J.len;
        uint32_t v = 0u;
        if (i >= J.z && i < J.z + J.h)
            v = J.src1[s * J.src1_stride + (i - J.z)];
        else if (i >= J.z + J.h)
            v = J.src2[s * J.src2_stride + J.src2_off + (i - J.z - J.h)];
        J.dst[s * J.dst_stride + i] = v;
    }
}

// ---------------------------------------------------------------------------
// History maintenance and small helpers
// ---------------------------------------------------------------------------

// For every stream s: dst[s*dst_stride + dst_off + i] = src[s*src_stride + src_off + i], i < bytes.
__global__ void copy_rows_kernel(uint8_t *__restrict__ dst, int64_t dst_stride, int64_t dst_off,
                                 const uint8_t *__restrict__ src, int64_t src_stride, int64_t src_off,
                                 int64_t bytes, int streams)
{
    const int64_t total = bytes * streams;
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
         e += int64_t(gridDim.x) * blockDim.x) {
        const int64_t s = e / bytes, i = e % bytes;
        dst[s * dst_stride + dst_off + i] = src[s * src_stride + src_off + i];
    }
}

__global__ void fill_zero_kernel(uint8_t *__restrict__ p, int64_t bytes, int *__restrict__ status)
{
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < bytes;
         e += int64_t(gridDim.x) * blockDim.x)
        p[e] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *status = 0;
}

__global__ void unpack_kernel(const uint8_t *__restrict__ raw, int64_t first, int64_t count,
                              int32_t *__restrict__ out)
{
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < count;
         e += int64_t(gridDim.x) * blockDim.x) {
        const int64_t j = first + e;
        // 64-bit safe form of sample10 for arbitrary offsets
        const int64_t bit = 10 * j;
        const uint32_t v = (uint32_t(raw[bit >> 3]) << 8) | uint32_t(raw[(bit >> 3) + 1]);
        out[e] = int32_t(v << (16u + uint32_t(bit & 7))) >> 22;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Static device scratch of fe_channelize_noalloc: the intermediate buffers of
// a call (filtered samples, int8 spectra before the corner turn, reordered
// gains, history assembly), FE_NOALLOC_SCRATCH_BYTES on every GPU the library
// runs on, held until the process ends.  In host code `scratch` names a
// host-side stand-in, not the device array: its device address comes from
// hipGetSymbolAddress, once per device (scratch_address), and only that
// address is ever handed to kernels.
// ---------------------------------------------------------------------------

static __device__ __align__(256) uint8_t scratch[FE_NOALLOC_SCRATCH_BYTES];

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

constexpr int EV_PER_CALL = 5;

struct fe_stream {
    int n, T, Tk, A, S, D, H;
    int prec;               // FE_PREC_*
    int fir_batches;        // FIR schedule: run length in batches of spectra (FP32) or
                            // tiles per chain (matrix-core FIR); 0: chosen per launch
    int path;               // FE_PATH_*: split or fused kernels (FP32, n <= 4096, T <= 16)
    int fft_parts;          // n > 8192: workgroups per spectrum of the post kernel (1..9); 0: per call
    float tap_scale;        // FP16 mode: taps scaled by 2^sc on the matrix cores
    float out_scale;        // 2^-sc, applied to the FIR's FP32 result
    int64_t max_samples;
    int device;
    int cus;                // compute units of the device
    hipStream_t stream;
    float *d_taps;          // [2n*Tk], zero-padded in front when Tk > T
    float2 *d_tw;           // FFT twiddle blocks
    float2 *d_untangle;     // exp(-i pi k / n) (n > 8192: in residue-plane order)
    float2 *d_gpl;          // n > 8192: the call's gains in residue-plane order, [A*2][n]
    float2 *d_tw16;         // matrix-stage twiddles [stage][group][16] (reduced modes)
    float2 *d_twf;          // n > 8192: first-level twiddles exp(-2 pi i gam d / n), [n/16][16]
    uint32_t *d_dfta;       // DFT-16 A-operand images [K half][hi, lo][lane][8 x 16 bit]
    uint8_t *d_hist;        // [A*2][H*5/4]
    uint8_t *d_hist_tmp;    // same, used when a call is shorter than H
    uint8_t *d_seam;        // FP32: staging of the FIR's seam, seam_bytes()
    float *d_g;             // [A*2][max_samples/(2n)][2n]
    uint32_t *d_spec8;      // [A*2][max_samples/(2n)][n] (re, im) int8 pairs
    int *d_status;
    // kernel timing (fe_stream_timing): EV_PER_CALL events per recorded call
    std::vector<hipEvent_t> ev;
    int ev_used;            // calls recorded since the last read
    bool timing;
};

namespace {

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

int kernel_taps(int T)
{
    static const int sup[] = {4, 8, 16, 24, 32};
    for (int t : sup)
        if (T <= t)
            return t;
    return -1;
}

template <int N>
std::vector<float2> make_twiddles()
{
    std::vector<float2> tw(size_t(tw_offset<N>(Plan<N>::P)) + 1);
    for (int p = 0; p < Plan<N>::P; ++p) {
        const int L = tw_L<N>(p), R = Plan<N>::R[p];
        if (L == 1)
            continue;
        const int off = tw_offset<N>(p);
        for (int j = 0; j < L; ++j)
            for (int q = 1; q < R; ++q) {
                // exp(-2 pi i j q / (L R)) from an exact integer angle index
                const long double a = -2.0L * 3.141592653589793238462643383279503L
                                      * (long double)((int64_t)j * q) / (long double)(L * R);
                tw[size_t(off) + size_t(q - 1) * L + j] =
                    make_float2(float(std::cos(a)), float(std::sin(a)));
            }
    }
    return tw;
}

std::vector<float2> twiddles_for(int n)
{
    switch (n) {
    case 256: return make_twiddles<256>();
    case 512: return make_twiddles<512>();
    case 1024: return make_twiddles<1024>();
    case 2048: return make_twiddles<2048>();
    case 4096: return make_twiddles<4096>();
    case 8192: return make_twiddles<8192>();
    case 16384: return make_twiddles<1024>();      // sub-transforms of n/16 points
    case 32768: return make_twiddles<2048>();
    default: return {};
    }
}

// Matrix-core FIR tap counts: one 32-row K-step holds 16 spectra x 16 taps,
// two hold up to 32 taps.
int kernel_taps_mfma(int T) { return T <= 16 ? 16 : 32; }

uint16_t f16_bits(float x)
{
    const _Float16 h = (_Float16)x;
    uint16_t u;
    std::memcpy(&u, &h, 2);
    return u;
}
float f16_value(uint16_t u)
{
    _Float16 h;
    std::memcpy(&h, &u, 2);
    return float(h);
}
uint16_t bf16_bits(float x)              // round to nearest even (finite x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}
float bf16_value(uint16_t b)
{
    const uint32_t u = uint32_t(b) << 16;
    float x;
    std::memcpy(&x, &u, 4);
    return x;
}

// A operand of the matrix stages: the real 32 x 32 form of the DFT-16 matrix
// W[d][j] = exp(-2 pi i dj/16), scaled by 1/4.  Row m < 16 gives Re Y_m, row
// 16 + m gives Im Y_m; column 2j + c takes Re x_j (c = 0) or Im x_j (c = 1).
// Lane l of K half kap holds A[l mod 32][16 kap + 8 (l div 32) + e], e < 8;
// in split mode a second image holds the BF16 residuals.
std::vector<uint32_t> make_dft_a(int prec)
{
    // DFT-16: [K half][hi, lo][lane][8 x 16 bit]; then DFT-32 (radix-32 last
    // stage): [row tile][K step][hi, lo][lane][8 x 16 bit]
    std::vector<uint32_t> img(size_t(2) * 2 * 64 * 4 + size_t(2) * 4 * 2 * 64 * 4, 0u);
    const long double pi = 3.141592653589793238462643383279503L;
    auto store = [&](size_t image_word, int e, double val) {
        uint16_t hi, lo = 0;
        if (prec == FE_PREC_FP16) {
            hi = f16_bits(float(val));
        } else {
            hi = bf16_bits(float(val));
            lo = bf16_bits(float(val - double(bf16_value(hi))));
        }
        img[image_word] |= uint32_t(hi) << (16 * (e % 2));
        img[image_word + 64 * 4] |= uint32_t(lo) << (16 * (e % 2));   // the lo image follows the hi one
    };
    const size_t base32 = size_t(2) * 2 * 64 * 4;
    for (int mt = 0; mt < 2; ++mt)
        for (int kap = 0; kap < 4; ++kap)
            for (int lane = 0; lane < 64; ++lane)
                for (int e = 0; e < 8; ++e) {
                    // row 32 mt + m: real (mt = 0) or imaginary (mt = 1) part of output d = m;
                    // column k: real (c = 0) or imaginary (c = 1) part of input j
                    const int m = lane % 32, kq = lane / 32;
                    const int k = 16 * kap + 8 * kq + e;
                    const int j = k / 2, c = k % 2, d = m;
                    const long double th = 2.0L * pi * (long double)((d * j) % 32) / 32.0L;
                    const long double cs = std::cos(th), sn = std::sin(th);
                    const double val = double(mt == 0 ? (c == 0 ? cs : sn) : (c == 0 ? -sn : cs));
                    store(base32 + (size_t((mt * 4 + kap) * 2) * 64 + lane) * 4 + e / 2, e, val);
                }
    for (int kap = 0; kap < 2; ++kap)
        for (int lane = 0; lane < 64; ++lane)
            for (int e = 0; e < 8; ++e) {
                const int m = lane % 32, kq = lane / 32;
                const int k = 16 * kap + 8 * kq + e;
                const int j = k / 2, c = k % 2, d = m % 16;
                const long double th = 2.0L * pi * (long double)((d * j) % 16) / 16.0L;
                const long double cs = std::cos(th), sn = std::sin(th);
                const double val = double(0.25L * (m < 16 ? (c == 0 ? cs : sn) : (c == 0 ? -sn : cs)));
                uint16_t hi, lo = 0;
                if (prec == FE_PREC_FP16) {
                    hi = f16_bits(float(val));
                } else {
                    hi = bf16_bits(float(val));
                    lo = bf16_bits(float(val - double(bf16_value(hi))));
                }
                for (int part = 0; part < 2; ++part) {
                    const uint16_t v = part == 0 ? hi : lo;
                    const size_t word = (size_t(kap * 2 + part) * 64 + lane) * 4 + e / 2;
                    img[word] |= uint32_t(v) << (16 * (e % 2));
                }
            }
    return img;
}

// Matrix-stage twiddles: entry [s][gam][d] = exp(-2 pi i (gam mod R') d / R_s).
// The table of the all-radix-16 plan; a plan ending in radix 32 uses its
// first stages (stage s's entries depend on n and s only).
template <int N>
std::vector<float2> make_tw16()
{
    constexpr int S16 = N >= 4096 ? 3 : 2, G = N / 16;
    std::vector<float2> tw(size_t(S16) * G * 16);
    const long double pi = 3.141592653589793238462643383279503L;
    for (int st = 0; st < S16; ++st) {
        const int rn = mstage_rn<N>(st), rs = 16 * rn;
        for (int gam = 0; gam < G; ++gam)
            for (int d = 0; d < 16; ++d) {
                const int64_t q = (int64_t(gam % rn) * d) % rs;
                const long double a = -2.0L * pi * (long double)q / (long double)rs;
                tw[(size_t(st) * G + gam) * 16 + d] = make_float2(float(std::cos(a)), float(std::sin(a)));
            }
    }
    return tw;
}

std::vector<float2> tw16_for(int n)
{
    switch (n) {
    case 256: return make_tw16<256>();
    case 512: return make_tw16<512>();
    case 1024: return make_tw16<1024>();
    case 2048: return make_tw16<2048>();
    case 4096: return make_tw16<4096>();
    case 8192: return make_tw16<8192>();
    default: return {};
    }
}

fe_status hip_status(hipError_t e) { return e == hipSuccess ? FE_OK : FE_EHIP; }

// Device address of the static scratch on `device`, which must be the
// current device: looked up once per device (at the first stream creation
// on it), NULL if the lookup failed.
constexpr int kMaxDevices = 64;
std::once_flag g_scratch_once[kMaxDevices];
uint8_t *g_scratch_ptr[kMaxDevices];

uint8_t *scratch_address(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return nullptr;
    std::call_once(g_scratch_once[device], [device]() {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_ptr[device] = e == hipSuccess ? static_cast<uint8_t *>(p) : nullptr;
        if (e != hipSuccess)
            (void)hipGetLastError();
    });
    return g_scratch_ptr[device];
}

bool matrix_fir(const fe_stream *s);
bool fused_path(const fe_stream *s);

// Per-call intermediate buffers of a call: the stream's own workspace, or
// the library's static scratch (fe_channelize_noalloc).
struct Work {
    float *g;               // filtered samples g (float32; FP16 streams store FP16)
    uint32_t *spec8;        // int8 spectra before the corner turn
    float2 *gpl;            // n > 8192: the call's gains in residue-plane order
    uint8_t *hist_tmp;      // history assembly for calls shorter than H
    uint8_t *seam;          // FP32 FIR: the history's tail and the chunk's first rows
};

unsigned grid_for(int64_t work, int threads)
{
    int64_t b = (work + threads - 1) / threads;
    if (b < 1)
        b = 1;
    if (b > 65536)
        b = 65536;
    return unsigned(b);
}

// The FIR's seam: the first T' - 1 + ceil(D / 2n) spectra of a call read
// rows before it (the history).  They are filtered from a staging buffer of
// ceil(H / 2n) history rows followed by the chunk's first rows, on the same
// grouped fast path as the rest of the call.
int seam_rows_before(const fe_stream *s) { return (s->H + 2 * s->n - 1) / (2 * s->n); }
int seam_spectra(const fe_stream *s) { return s->Tk - 1 + (s->D + 2 * s->n - 1) / (2 * s->n); }
int64_t seam_bytes(const fe_stream *s)
{
    return int64_t(2 * s->A) * (seam_rows_before(s) + seam_spectra(s)) * (int64_t(2 * s->n) * 5 / 4);
}

template <int T, int GM>
void launch_fir_range(const fe_stream *s, const uint8_t *raw, int64_t raw_stride, int mrows, int moff, int M,
                      const double *delays, void *g, int mb, int me, bool front = false)
{
    const int n2 = 2 * s->n;
    const int streams = 2 * s->A;
    const int colblocks = n2 / (2 * FIR_THREADS);            // a column pair per thread
    // runs of R spectra (whole batches of B = (64/T)T); longer runs load the
    // taps less often, shorter ones give more workgroups
    constexpr int B = (64 / T) * T;
    int R = 4 * B;
    if (s->fir_batches > 0)
        R = s->fir_batches * B;                  // set by fe_stream_autotune
    else
        while (R > B && int64_t(streams) * ((me - mb + R - 1) / R) * colblocks < 2048)
            R -= B;
    const int runs = (me - mb + R - 1) / R;
    const int64_t blocks = int64_t(streams) * runs * colblocks;
    if constexpr ((GM == G_F32 || GM == G_F16) && T <= 16) {
        if (front) {
            hipLaunchKernelGGL((fir_kernel<T, GM, true>), dim3(unsigned(blocks)), dim3(FIR_THREADS), 0, s->stream,
                               raw, raw_stride, s->d_hist, int64_t(s->H) * 5 / 4, s->H, s->d_taps, delays, g,
                               n2, M, s->D, R, colblocks, runs, mb, me, moff, mrows, s->d_twf);
            return;
        }
    }
    hipLaunchKernelGGL((fir_kernel<T, GM>), dim3(unsigned(blocks)), dim3(FIR_THREADS), 0, s->stream,
                       raw, raw_stride, s->d_hist, int64_t(s->H) * 5 / 4, s->H, s->d_taps, delays, g,
                       n2, M, s->D, R, colblocks, runs, mb, me, moff, mrows, nullptr);
}

template <int T, int GM>
void launch_fir_T(const fe_stream *s, const Work &wk, const uint8_t *raw, int64_t N, const double *delays,
                  void *g, int mb, int me, bool front = false)
{
    const int n2 = 2 * s->n;
    const int M = int(N / n2);
    const int S0 = std::min(me, seam_spectra(s));
    int main_mb = mb;
    if (mb < S0) {
        const int K = seam_rows_before(s);
        const int rows = K + S0;
        const int64_t row_bytes = int64_t(n2) * 5 / 4;             // a multiple of 4
        const int64_t dst_words = rows * row_bytes / 4;
        const int64_t zero_words = (int64_t(K) * n2 - s->H) * 5 / 16;
        const int64_t hist_words = int64_t(s->H) * 5 / 16;
        const int streams = 2 * s->A;
        hipLaunchKernelGGL(seam_stage_kernel, dim3(grid_for(dst_words * streams, 256)), dim3(256), 0, s->stream,
                           reinterpret_cast<uint32_t *>(wk.seam), dst_words,
                           reinterpret_cast<const uint32_t *>(s->d_hist), hist_words,
                           reinterpret_cast<const uint32_t *>(raw), N * 5 / 16, zero_words,
                           int64_t(S0) * row_bytes / 4, streams);
        launch_fir_range<T, GM>(s, wk.seam, rows * row_bytes, rows, K, M, delays, g, K + mb, K + S0, front);
        main_mb = S0;
    }
    if (main_mb < me)
        launch_fir_range<T, GM>(s, raw, N * 5 / 4, M, 0, M, delays, g, main_mb, me, front);
}

template <int TK, int PREC>
void launch_fir_mfma_T(const fe_stream *s, const uint8_t *raw, int64_t N, const double *delays,
                       void *g, bool g_f32, int mb, int me)
{
    const int n2 = 2 * s->n;
    const int M = int(N / n2);
    const int ctiles = n2 / FM_COLS;
    const int ftiles = (me - mb + FM_SPEC - 1) / FM_SPEC;
    // chains of consecutive spectrum tiles per workgroup (the taps are
    // loaded once per chain and each tile's rows are fetched during the
    // previous tile's contraction); about 1024 workgroups, two per CU
    const int64_t tiles = int64_t(2 * s->A) * ftiles * ctiles;
    int chain = int(std::min<int64_t>(ftiles, std::max<int64_t>(1, tiles / 1024)));
    if (s->fir_batches > 0)
        chain = std::min(ftiles, s->fir_batches);           // set by fe_stream_autotune
    const int64_t blocks = int64_t(2 * s->A) * ((ftiles + chain - 1) / chain) * ctiles;
    if (PREC == FE_PREC_FP16 && !g_f32)
        hipLaunchKernelGGL((fir_mfma_kernel<TK, PREC, GOUT_F16>), dim3(unsigned(blocks)), dim3(256), 0,
                           s->stream, raw, N * 5 / 4, N, s->d_hist, int64_t(s->H) * 5 / 4, s->H, s->d_taps,
                           s->tap_scale, s->out_scale, delays, g, n2, M, s->D, mb, me, ctiles, ftiles, chain);
    else
        hipLaunchKernelGGL((fir_mfma_kernel<TK, PREC, GOUT_F32>), dim3(unsigned(blocks)), dim3(256), 0,
                           s->stream, raw, N * 5 / 4, N, s->d_hist, int64_t(s->H) * 5 / 4, s->H, s->d_taps,
                           s->tap_scale, s->out_scale, delays, g, n2, M, s->D, mb, me, ctiles, ftiles, chain);
}

template <int GM>
void launch_fir_vec(const fe_stream *s, const Work &wk, const uint8_t *raw, int64_t N, const double *delays, void *g,
                    int mb, int me, bool front = false)
{
    switch (s->Tk) {
    case 4: launch_fir_T<4, GM>(s, wk, raw, N, delays, g, mb, me, front); break;
    case 8: launch_fir_T<8, GM>(s, wk, raw, N, delays, g, mb, me, front); break;
    case 16: launch_fir_T<16, GM>(s, wk, raw, N, delays, g, mb, me, front); break;
    case 24: launch_fir_T<24, GM>(s, wk, raw, N, delays, g, mb, me, front); break;
    case 32: launch_fir_T<32, GM>(s, wk, raw, N, delays, g, mb, me, front); break;
    }
}

// Whether a call's FIR also does the first FFT stage (FP32 and FP16
// streams, n > 8192, up to 16 taps -- with more, the FIR's window and the
// DFT do not fit the registers together -- and not for the FIR-stage output
// of fe_channelize_fir).
bool fir_fronts(const fe_stream *s, bool g_out)
{
    return (s->prec == FE_PREC_FP32 || s->prec == FE_PREC_FP16) && s->n > 8192 && s->Tk <= 16 && !g_out;
}

void launch_fir(const fe_stream *s, const Work &wk, const uint8_t *raw, int64_t N, const double *delays, float *g,
                int mb, int me, bool g_out = false)
{
    if (s->prec != FE_PREC_FP32 && !matrix_fir(s)) {
        // reduced-precision streams on the vector FIR: float32 arithmetic;
        // FP16 streams store FP16 (the matrix-core FFT's operand; above 8192
        // channels the float32 two-level FFT's input), BF16 streams float32
        // (their FFT splits it into hi + lo)
        if (s->prec == FE_PREC_FP16 && g_out)
            launch_fir_vec<G_F32_AS_F16>(s, wk, raw, N, delays, g, mb, me);
        else if (s->prec == FE_PREC_FP16)
            launch_fir_vec<G_F16>(s, wk, raw, N, delays, g, mb, me, fir_fronts(s, g_out));
        else
            launch_fir_vec<G_F32>(s, wk, raw, N, delays, g, mb, me);
        return;
    }
    if (s->prec != FE_PREC_FP32) {
        if (s->prec == FE_PREC_FP16) {
            if (s->Tk == 16)
                launch_fir_mfma_T<16, FE_PREC_FP16>(s, raw, N, delays, g, g_out, mb, me);
            else
                launch_fir_mfma_T<32, FE_PREC_FP16>(s, raw, N, delays, g, g_out, mb, me);
        } else {
            if (s->Tk == 16)
                launch_fir_mfma_T<16, FE_PREC_BF16>(s, raw, N, delays, g, g_out, mb, me);
            else
                launch_fir_mfma_T<32, FE_PREC_BF16>(s, raw, N, delays, g, g_out, mb, me);
        }
        return;
    }
    launch_fir_vec<G_F32>(s, wk, raw, N, delays, g, mb, me, fir_fronts(s, g_out));
}

template <int N>
void launch_post_N(const fe_stream *s, const Work &wk, int M, const double *delays, const double *phases,
                   const float *gains, float *y_out, int mb, int me)
{
    const unsigned blocks = unsigned(s->A * (me - mb) * 2);
    if (y_out)
        hipLaunchKernelGGL((fft_post_kernel<N, OUT_PREQUANT>), dim3(blocks), dim3(N / 16), 0, s->stream,
                           wk.g, delays, phases, reinterpret_cast<const float2 *>(gains), s->d_tw,
                           s->d_untangle, wk.spec8, reinterpret_cast<float2 *>(y_out), s->d_status,
                           M, s->D, mb, me);
    else
        hipLaunchKernelGGL((fft_post_kernel<N, OUT_INT8>), dim3(blocks), dim3(N / 16), 0, s->stream,
                           wk.g, delays, phases, reinterpret_cast<const float2 *>(gains), s->d_tw,
                           s->d_untangle, wk.spec8, reinterpret_cast<float2 *>(y_out), s->d_status,
                           M, s->D, mb, me);
}

// Kernel 2H in place of kernels 2 and 3 (FP32, n <= 8192, int8 output)
template <int N>
void launch_post_heap_N(const fe_stream *s, const Work &wk, int M, const double *delays, const double *phases,
                        const float *gains, int8_t *out)
{
    if (s->S % 2 == 0)
        hipLaunchKernelGGL((fft_post_heap_kernel<N, 2>), dim3(unsigned(s->A * (M / 2))), dim3(N / 16), 0,
                           s->stream, wk.g, delays, phases, reinterpret_cast<const float2 *>(gains), s->d_tw,
                           s->d_untangle, out, s->d_status, M, s->D, s->S);
    else
        hipLaunchKernelGGL((fft_post_heap_kernel<N, 1>), dim3(unsigned(s->A * M)), dim3(N / 16), 0,
                           s->stream, wk.g, delays, phases, reinterpret_cast<const float2 *>(gains), s->d_tw,
                           s->d_untangle, out, s->d_status, M, s->D, s->S);
}

// Whether a call of M spectra runs the folded FFT/post kernel (kernel 2H, or
// 2MH for FP16/BF16 streams on the vector FIR).  FE_PATH_AUTO folds FP32
// calls only, and only when the folded launch (a workgroup per antenna and
// run of one or two spectra) still gives every CU eight workgroups: on
// fewer it is slower than the split kernel's workgroup per spectrum and
// polarization plus the separate turn.  (Kernel 2MH measures as fast as 2M
// plus the turn, not faster: 0.212 against 0.161 + 0.049 ms for FP16 at
// 4096 channels; fe_stream_autotune times both.)
bool heap_fold(const fe_stream *s, int M)
{
    if (s->n > 8192 || fused_path(s) || matrix_fir(s))
        return false;
    if (s->path == FE_PATH_SPLIT_FOLDED)
        return true;
    if (s->prec != FE_PREC_FP32)
        return false;
    const int spw = s->S % 2 == 0 ? 2 : 1;
    return s->path == FE_PATH_AUTO && int64_t(s->A) * (M / spw) >= int64_t(8) * s->cus;
}

// Kernel 2MH in place of kernels 2M and 3
template <int N, int PREC>
void launch_post_mfma_heap_N(const fe_stream *s, const Work &wk, int M, const double *delays,
                             const double *phases, const float *gains, int8_t *out)
{
    const u32x4 *dfta = reinterpret_cast<const u32x4 *>(s->d_dfta);
    const float2 *gn = reinterpret_cast<const float2 *>(gains);
    if (s->S % 2 == 0)
        hipLaunchKernelGGL((fft_mfma_heap_kernel<N, PREC, 2>), dim3(unsigned(s->A * (M / 2))),
                           dim3(MPlan<N, PREC>::NT), 0, s->stream, wk.g, delays, phases, gn, s->d_tw16, s->d_untangle,
                           dfta, out, s->d_status, M, s->D, s->S);
    else
        hipLaunchKernelGGL((fft_mfma_heap_kernel<N, PREC, 1>), dim3(unsigned(s->A * M)), dim3(MPlan<N, PREC>::NT), 0,
                           s->stream, wk.g, delays, phases, gn, s->d_tw16, s->d_untangle, dfta, out,
                           s->d_status, M, s->D, s->S);
}

template <int PREC>
void launch_post_mfma_heap(const fe_stream *s, const Work &wk, int M, const double *delays, const double *phases,
                           const float *gains, int8_t *out)
{
    switch (s->n) {
    case 256: launch_post_mfma_heap_N<256, PREC>(s, wk, M, delays, phases, gains, out); break;
    case 512: launch_post_mfma_heap_N<512, PREC>(s, wk, M, delays, phases, gains, out); break;
    case 1024: launch_post_mfma_heap_N<1024, PREC>(s, wk, M, delays, phases, gains, out); break;
    case 2048: launch_post_mfma_heap_N<2048, PREC>(s, wk, M, delays, phases, gains, out); break;
    case 4096: launch_post_mfma_heap_N<4096, PREC>(s, wk, M, delays, phases, gains, out); break;
    case 8192: launch_post_mfma_heap_N<8192, PREC>(s, wk, M, delays, phases, gains, out); break;
    }
}

void launch_post_heap(const fe_stream *s, const Work &wk, int M, const double *delays, const double *phases,
                      const float *gains, int8_t *out)
{
    if (s->prec == FE_PREC_FP16) {
        launch_post_mfma_heap<FE_PREC_FP16>(s, wk, M, delays, phases, gains, out);
        return;
    }
    if (s->prec == FE_PREC_BF16) {
        launch_post_mfma_heap<FE_PREC_BF16>(s, wk, M, delays, phases, gains, out);
        return;
    }
    switch (s->n) {
    case 256: launch_post_heap_N<256>(s, wk, M, delays, phases, gains, out); break;
    case 512: launch_post_heap_N<512>(s, wk, M, delays, phases, gains, out); break;
    case 1024: launch_post_heap_N<1024>(s, wk, M, delays, phases, gains, out); break;
    case 2048: launch_post_heap_N<2048>(s, wk, M, delays, phases, gains, out); break;
    case 4096: launch_post_heap_N<4096>(s, wk, M, delays, phases, gains, out); break;
    case 8192: launch_post_heap_N<8192>(s, wk, M, delays, phases, gains, out); break;
    }
}

template <int N, int PREC>
void launch_post_mfma_N(const fe_stream *s, const Work &wk, int M, const double *delays, const double *phases,
                        const float *gains, float *y_out, int mb, int me)
{
    const unsigned blocks = unsigned(s->A * (me - mb) * 2);
    const u32x4 *dfta = reinterpret_cast<const u32x4 *>(s->d_dfta);
    if (y_out)
        hipLaunchKernelGGL((fft_mfma_kernel<N, PREC, OUT_PREQUANT>), dim3(blocks), dim3(MPlan<N, PREC>::NT), 0,
                           s->stream, wk.g, delays, phases, reinterpret_cast<const float2 *>(gains),
                           s->d_tw16, s->d_untangle, dfta, wk.spec8, reinterpret_cast<float2 *>(y_out),
                           s->d_status, M, s->D, mb, me);
    else
        hipLaunchKernelGGL((fft_mfma_kernel<N, PREC, OUT_INT8>), dim3(blocks), dim3(MPlan<N, PREC>::NT), 0,
                           s->stream, wk.g, delays, phases, reinterpret_cast<const float2 *>(gains),
                           s->d_tw16, s->d_untangle, dfta, wk.spec8, reinterpret_cast<float2 *>(y_out),
                           s->d_status, M, s->D, mb, me);
}

template <int PREC>
void launch_post_mfma(const fe_stream *s, const Work &wk, int M, const double *delays, const double *phases,
                      const float *gains, float *y_out, int mb, int me)
{
    switch (s->n) {
    case 256: launch_post_mfma_N<256, PREC>(s, wk, M, delays, phases, gains, y_out, mb, me); break;
    case 512: launch_post_mfma_N<512, PREC>(s, wk, M, delays, phases, gains, y_out, mb, me); break;
    case 1024: launch_post_mfma_N<1024, PREC>(s, wk, M, delays, phases, gains, y_out, mb, me); break;
    case 2048: launch_post_mfma_N<2048, PREC>(s, wk, M, delays, phases, gains, y_out, mb, me); break;
    case 4096: launch_post_mfma_N<4096, PREC>(s, wk, M, delays, phases, gains, y_out, mb, me); break;
    case 8192: launch_post_mfma_N<8192, PREC>(s, wk, M, delays, phases, gains, y_out, mb, me); break;
    }
}

template <int NL>
void launch_post_large(const fe_stream *s, const Work &wk, int M, const double *delays, const double *phases,
                       const float *gains, float *y_out, int mb, int me, bool fronted)
{
    if (fronted) {
        // the FIR did the first stage: only the gains' reordering is left
        const int64_t total = int64_t(s->A) * 2 * NL;
        hipLaunchKernelGGL(gains_planes_kernel, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s->stream,
                           reinterpret_cast<const float2 *>(gains), wk.gpl, NL, total);
    } else {
        const int64_t fthreads = int64_t(s->A) * 2 * (me - mb) * (NL / 16);
        if (s->prec == FE_PREC_FP16)
            hipLaunchKernelGGL(fft_front_kernel<true>, dim3(unsigned((fthreads + 255) / 256)), dim3(256), 0,
                               s->stream, wk.g, s->d_twf, reinterpret_cast<const float2 *>(gains), wk.gpl, NL, M,
                               mb, me, s->A);
        else
            hipLaunchKernelGGL(fft_front_kernel<false>, dim3(unsigned((fthreads + 255) / 256)), dim3(256), 0,
                               s->stream, wk.g, s->d_twf, reinterpret_cast<const float2 *>(gains), wk.gpl, NL, M,
                               mb, me, s->A);
    }
    // the nine rounds of each spectrum (pol) over 9 workgroups for calls of
    // under 128 spectra-pols, over 3 under 512, else one workgroup (measured
    // at 32768 channels: 128 items 0.074 -> 0.047 ms with 3 parts, 512 items
    // 0.130 ms with one part against 0.142 with 9)
    const int items = s->A * (me - mb) * 2;
    const int rparts = s->fft_parts > 0 ? s->fft_parts : items < 128 ? 9 : items < 512 ? 3 : 1;
    const unsigned blocks = unsigned(items * rparts);
    // FP16 streams hand the FFT its input as FP16 pairs (the two-level FFT
    // itself runs in float32)
    const bool f16 = s->prec == FE_PREC_FP16;
    if (y_out && f16)
        hipLaunchKernelGGL((fft_post_large_kernel<NL, OUT_PREQUANT, true>), dim3(blocks), dim3(NL / 128), 0,
                           s->stream, wk.g, delays, phases, wk.gpl, s->d_tw,
                           s->d_untangle, wk.spec8, reinterpret_cast<float2 *>(y_out), s->d_status, M, s->D,
                           mb, me, rparts);
    else if (y_out)
        hipLaunchKernelGGL((fft_post_large_kernel<NL, OUT_PREQUANT>), dim3(blocks), dim3(NL / 128), 0,
                           s->stream, wk.g, delays, phases, wk.gpl, s->d_tw,
                           s->d_untangle, wk.spec8, reinterpret_cast<float2 *>(y_out), s->d_status, M, s->D,
                           mb, me, rparts);
    else if (f16)
        hipLaunchKernelGGL((fft_post_large_kernel<NL, OUT_INT8, true>), dim3(blocks), dim3(NL / 128), 0,
                           s->stream, wk.g, delays, phases, wk.gpl, s->d_tw,
                           s->d_untangle, wk.spec8, reinterpret_cast<float2 *>(y_out), s->d_status, M, s->D,
                           mb, me, rparts);
    else
        hipLaunchKernelGGL((fft_post_large_kernel<NL, OUT_INT8>), dim3(blocks), dim3(NL / 128), 0,
                           s->stream, wk.g, delays, phases, wk.gpl, s->d_tw,
                           s->d_untangle, wk.spec8, reinterpret_cast<float2 *>(y_out), s->d_status, M, s->D,
                           mb, me, rparts);
}

void launch_post(const fe_stream *s, const Work &wk, int M, const double *delays, const double *phases,
                 const float *gains, float *y_out, int mb, int me, bool fronted = false)
{
    if (s->n == 16384) {
        launch_post_large<16384>(s, wk, M, delays, phases, gains, y_out, mb, me, fronted);
        return;
    }
    if (s->n == 32768) {
        launch_post_large<32768>(s, wk, M, delays, phases, gains, y_out, mb, me, fronted);
        return;
    }
    if (s->prec == FE_PREC_FP16) {
        launch_post_mfma<FE_PREC_FP16>(s, wk, M, delays, phases, gains, y_out, mb, me);
        return;
    }
    if (s->prec == FE_PREC_BF16) {
        launch_post_mfma<FE_PREC_BF16>(s, wk, M, delays, phases, gains, y_out, mb, me);
        return;
    }
    switch (s->n) {
    case 256: launch_post_N<256>(s, wk, M, delays, phases, gains, y_out, mb, me); break;
    case 512: launch_post_N<512>(s, wk, M, delays, phases, gains, y_out, mb, me); break;
    case 1024: launch_post_N<1024>(s, wk, M, delays, phases, gains, y_out, mb, me); break;
    case 2048: launch_post_N<2048>(s, wk, M, delays, phases, gains, y_out, mb, me); break;
    case 4096: launch_post_N<4096>(s, wk, M, delays, phases, gains, y_out, mb, me); break;
    case 8192: launch_post_N<8192>(s, wk, M, delays, phases, gains, y_out, mb, me); break;
    }
}

// The fused path (pfb_fused_kernel) can run FP32 streams with n <= 4096 and
// at most 16 (kernel) taps.  Chosen by default where it measured faster on
// MI355X than the split path (FIR kernel, g in device memory, FFT/post
// kernel): 8 taps or fewer and n <= 2048.  With 16 taps the fused kernel's
// FIR reloads every tap and re-unpacks T + 3 rows for each step of four
// spectra, where the split FIR keeps taps and a sliding window in registers.
bool fused_eligible(const fe_stream *s)
{
    return s->prec == FE_PREC_FP32 && s->n <= 4096 && s->Tk <= 16;
}

// FP16/BF16 streams: the FIR on the matrix cores (the banded Toeplitz
// contraction of fir_mfma_kernel) when chosen; by default the vector FIR
// (float32 arithmetic), which measured faster on MI355X -- the FIR is bound
// by memory traffic, and its Toeplitz form spends half the contraction on
// zeros and its staging on LDS bank conflicts.
bool matrix_fir(const fe_stream *s)
{
    return s->prec != FE_PREC_FP32 && s->path == FE_PATH_MATRIX_FIR && s->n <= 8192;
}

bool fused_path(const fe_stream *s)
{
    if (!fused_eligible(s) || s->path == FE_PATH_SPLIT || s->path == FE_PATH_MATRIX_FIR)
        return false;
    return s->path == FE_PATH_FUSED || (s->Tk <= 8 && s->n <= 2048);
}


// Workgroups of the fused kernel: a multiple of 8 (one share per XCD), at
// most what the GPU holds at once (s->fir_batches, when tuned, sets the
// workgroups per CU), never more than the work units.
unsigned fused_blocks(const fe_stream *s, int n, int64_t units)
{
    // resident workgroups per CU: LDS (4 spectra of n + n/16 complex values
    // and their phase tables) and at most 2048 threads per CU
    const int64_t lds = int64_t(PF_S) * (n + n / 16) * 8 + int64_t(PF_S) * (std::max(n / 64, 1) + 64) * 8;
    int per_cu = int(std::min<int64_t>(160 * 1024 / lds, 2048 / (n / 4)));
    if (s->fir_batches > 0)
        per_cu = std::min(per_cu, s->fir_batches);
    int64_t b = int64_t(std::max(per_cu, 1)) * s->cus;
    b = std::min<int64_t>(b, (units + 7) / 8 * 8);
    return unsigned(std::max<int64_t>(8, b / 8 * 8));
}

template <int N, int T>
void launch_fused_NT(const fe_stream *s, const Work &wk, const uint8_t *raw, int64_t Ns, const double *delays,
                     const double *phases, const float *gains, float *y_out, float *g_out, int mb, int me)
{
    const int M = int(Ns / (2 * N));
    const int nsteps = (me - mb + PF_S - 1) / PF_S;
    const int streams = 2 * s->A;
    const unsigned blocks = fused_blocks(s, N, int64_t(streams) * nsteps);
    const float2 *gn = reinterpret_cast<const float2 *>(gains);
    float2 *y2 = reinterpret_cast<float2 *>(y_out);
    float2 *g2 = reinterpret_cast<float2 *>(g_out);
    const int64_t rstride = Ns * 5 / 4, hstride = int64_t(s->H) * 5 / 4;
    if (g_out)
        hipLaunchKernelGGL((pfb_fused_kernel<N, T, OUT_G>), dim3(blocks), dim3(N / 4), 0, s->stream,
                           raw, rstride, s->d_hist, hstride, s->H, s->d_taps, delays, phases, gn, s->d_tw,
                           s->d_untangle, wk.spec8, y2, g2, s->d_status, M, s->D, streams, mb, me);
    else if (y_out)
        hipLaunchKernelGGL((pfb_fused_kernel<N, T, OUT_PREQUANT>), dim3(blocks), dim3(N / 4), 0, s->stream,
                           raw, rstride, s->d_hist, hstride, s->H, s->d_taps, delays, phases, gn, s->d_tw,
                           s->d_untangle, wk.spec8, y2, g2, s->d_status, M, s->D, streams, mb, me);
    else
        hipLaunchKernelGGL((pfb_fused_kernel<N, T, OUT_INT8>), dim3(blocks), dim3(N / 4), 0, s->stream,
                           raw, rstride, s->d_hist, hstride, s->H, s->d_taps, delays, phases, gn, s->d_tw,
                           s->d_untangle, wk.spec8, y2, g2, s->d_status, M, s->D, streams, mb, me);
}

template <int N>
void launch_fused_N(const fe_stream *s, const Work &wk, const uint8_t *raw, int64_t Ns, const double *delays,
                    const double *phases, const float *gains, float *y_out, float *g_out, int mb, int me)
{
    switch (s->Tk) {
    case 4: launch_fused_NT<N, 4>(s, wk, raw, Ns, delays, phases, gains, y_out, g_out, mb, me); break;
    case 8: launch_fused_NT<N, 8>(s, wk, raw, Ns, delays, phases, gains, y_out, g_out, mb, me); break;
    case 16: launch_fused_NT<N, 16>(s, wk, raw, Ns, delays, phases, gains, y_out, g_out, mb, me); break;
    }
}

void launch_fused(const fe_stream *s, const Work &wk, const uint8_t *raw, int64_t Ns, const double *delays,
                  const double *phases, const float *gains, float *y_out, float *g_out, int mb, int me)
{
    switch (s->n) {
    case 256: launch_fused_N<256>(s, wk, raw, Ns, delays, phases, gains, y_out, g_out, mb, me); break;
    case 512: launch_fused_N<512>(s, wk, raw, Ns, delays, phases, gains, y_out, g_out, mb, me); break;
    case 1024: launch_fused_N<1024>(s, wk, raw, Ns, delays, phases, gains, y_out, g_out, mb, me); break;
    case 2048: launch_fused_N<2048>(s, wk, raw, Ns, delays, phases, gains, y_out, g_out, mb, me); break;
    case 4096: launch_fused_N<4096>(s, wk, raw, Ns, delays, phases, gains, y_out, g_out, mb, me); break;
    }
}

void launch_corner_turn(const fe_stream *s, const Work &wk, int M, int8_t *out)
{
    const int ftiles = (M + CT - 1) / CT, ktiles = s->n / CT;
    // the two-level FFT (n > 8192, FP32) leaves its spectra as 16 residue planes
    const int ns = s->n > 8192 ? s->n / 16 : 0;
    hipLaunchKernelGGL(corner_turn_kernel, dim3(unsigned(s->A * ftiles * ktiles)), dim3(256), 0,
                       s->stream, wk.spec8, out, M, s->n, s->S, ftiles, ktiles, ns);
}

void launch_history_update(const fe_stream *s, const Work &wk, const uint8_t *raw, int64_t N)
{
    const int streams = 2 * s->A;
    const int64_t hb = int64_t(s->H) * 5 / 4;     // history bytes per stream
    const int64_t nb = N * 5 / 4;                 // chunk bytes per stream
    if (N >= s->H) {
        hipLaunchKernelGGL(copy_rows_kernel, dim3(grid_for(hb * streams, 256)), dim3(256), 0, s->stream,
                           s->d_hist, hb, int64_t(0), raw, nb, nb - hb, hb, streams);
    } else {
        // new history = old[N:] ++ chunk, assembled in the spare buffer first
        const int64_t keep = hb - nb;
        hipLaunchKernelGGL(copy_rows_kernel, dim3(grid_for(keep * streams, 256)), dim3(256), 0, s->stream,
                           wk.hist_tmp, hb, int64_t(0), s->d_hist, hb, nb, keep, streams);
        hipLaunchKernelGGL(copy_rows_kernel, dim3(grid_for(nb * streams, 256)), dim3(256), 0, s->stream,
                           wk.hist_tmp, hb, keep, raw, nb, int64_t(0), nb, streams);
        hipLaunchKernelGGL(copy_rows_kernel, dim3(grid_for(hb * streams, 256)), dim3(256), 0, s->stream,
                           s->d_hist, hb, int64_t(0), wk.hist_tmp, hb, int64_t(0), hb, streams);
    }
}

fe_status check_call(const fe_stream *s, const uint8_t *raw, int64_t N, const double *delays)
{
    if (!s || !raw || !delays)
        return FE_EINVAL;
    const int64_t unit = int64_t(2) * s->n * s->S;
    if (N <= 0 || N % unit)
        return FE_EINVAL;
    if (N > s->max_samples)
        return FE_ESIZE;
    return FE_OK;
}

// Bytes of static scratch a call of N samples needs (fe_channelize_noalloc):
// the regions of Work, each rounded up to 256 bytes.
int64_t scratch_need(const fe_stream *s, int64_t N, int64_t *off_spec8, int64_t *off_gpl, int64_t *off_hist,
                     int64_t *off_seam)
{
    auto up = [](int64_t b) { return (b + 255) / 256 * 256; };
    const int64_t streams = 2 * int64_t(s->A);
    const bool fused = fused_path(s);
    const int64_t g = fused ? 0 : up(streams * N * 4);
    const int64_t spec8 = up(streams * N);
    const int64_t gpl = s->n > 8192 ? up(streams * s->n * 8) : 0;
    const int64_t hist = N < s->H ? up(streams * (int64_t(s->H) * 5 / 4)) : 0;
    const int64_t seam = !fused && !matrix_fir(s) ? up(seam_bytes(s)) : 0;
    *off_spec8 = g;
    *off_gpl = g + spec8;
    *off_hist = g + spec8 + gpl;
    *off_seam = g + spec8 + gpl + hist;
    return g + spec8 + gpl + hist + seam;
}

fe_status channelize_impl(fe_stream *s, const uint8_t *raw, int64_t N, const double *delays,
                          const double *phases, const float *gains, int8_t *out, float *y_out,
                          float *g_out, uint8_t *scratch_base = nullptr)
{
    fe_status st = check_call(s, raw, N, delays);
    if (st != FE_OK)
        return st;
    if (!g_out && (!phases || !gains || (!out && !y_out)))
        return FE_EINVAL;
    Work wk = {s->d_g, s->d_spec8, s->d_gpl, s->d_hist_tmp, s->d_seam};
    if (scratch_base) {
        // the static scratch in place of the stream's workspace
        int64_t o_spec8, o_gpl, o_hist, o_seam;
        if (scratch_need(s, N, &o_spec8, &o_gpl, &o_hist, &o_seam) > int64_t(FE_NOALLOC_SCRATCH_BYTES))
            return FE_ESIZE;
        wk.g = reinterpret_cast<float *>(scratch_base);
        wk.spec8 = reinterpret_cast<uint32_t *>(scratch_base + o_spec8);
        wk.gpl = reinterpret_cast<float2 *>(scratch_base + o_gpl);
        wk.hist_tmp = scratch_base + o_hist;
        wk.seam = scratch_base + o_seam;
    }
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess)
        return FE_EHIP;
    if (cur != s->device && hipSetDevice(s->device) != hipSuccess)
        return FE_EHIP;
    (void)hipGetLastError();
    const int M = int(N / (2 * s->n));
    hipEvent_t *ev = nullptr;
    if (s->timing && size_t(s->ev_used + 1) * EV_PER_CALL <= s->ev.size())
        ev = &s->ev[size_t(s->ev_used++) * EV_PER_CALL];
    auto mark = [&](int i) {
        if (ev)
            (void)hipEventRecord(ev[i], s->stream);
    };
    mark(0);
    const bool fused = fused_path(s);
    if (fused)
        launch_fused(s, wk, raw, N, delays, phases, gains, y_out, g_out, 0, M);
    else
        launch_fir(s, wk, raw, N, delays, g_out ? g_out : wk.g, 0, M, g_out != nullptr);
    mark(1);
    launch_history_update(s, wk, raw, N);
    mark(2);
    // int8 output on the FP32 split path: the FFT/post kernel writes the heaps
    const bool heap = !g_out && !y_out && !fused && heap_fold(s, M);
    if (heap)
        launch_post_heap(s, wk, M, delays, phases, gains, out);
    else if (!g_out && !fused)
        launch_post(s, wk, M, delays, phases, gains, y_out, 0, M, fir_fronts(s, false));
    mark(3);
    if (!g_out && !y_out && !heap)
        launch_corner_turn(s, wk, M, out);
    mark(4);
    st = hip_status(hipGetLastError());
    if (cur != s->device)
        (void)hipSetDevice(cur);
    return st;
}

void free_events(fe_stream *s)
{
    for (hipEvent_t e : s->ev)
        (void)hipEventDestroy(e);
    s->ev.clear();
    s->ev_used = 0;
    s->timing = false;
}

void free_stream(fe_stream *s)
{
    if (!s)
        return;
    free_events(s);
    (void)hipFree(s->d_taps);
    (void)hipFree(s->d_tw);
    (void)hipFree(s->d_untangle);
    (void)hipFree(s->d_gpl);
    (void)hipFree(s->d_tw16);
    (void)hipFree(s->d_twf);
    (void)hipFree(s->d_dfta);
    (void)hipFree(s->d_hist);
    (void)hipFree(s->d_hist_tmp);
    (void)hipFree(s->d_seam);
    (void)hipFree(s->d_g);
    (void)hipFree(s->d_spec8);
    (void)hipFree(s->d_status);
    delete s;
}

}  // namespace

extern "C" {

fe_status fe_stream_create(const fe_config *cfg, void *hip_stream, fe_stream **out)
{
    if (!cfg || !out || !cfg->weights)
        return FE_EINVAL;
    if (cfg->precision != FE_PREC_FP32 && cfg->precision != FE_PREC_FP16 && cfg->precision != FE_PREC_BF16)
        return FE_EINVAL;
    const int n = cfg->n_channels, T = cfg->taps;
    if (!is_pow2(n) || n < 256 || n > 32768 || (n > 8192 && cfg->precision == FE_PREC_BF16)
        || T < 1 || T > 32 || cfg->n_antennas < 1
        || cfg->spectra_per_heap < 1 || cfg->max_delay < 0 || cfg->max_samples <= 0)
        return FE_EINVAL;
    const int64_t unit = int64_t(2) * n * cfg->spectra_per_heap;
    if (cfg->max_samples % unit || cfg->max_samples > (int64_t(1) << 28))
        return FE_EINVAL;
    if (int64_t(cfg->max_delay) > (int64_t(1) << 24))
        return FE_EINVAL;

    fe_stream *s = new (std::nothrow) fe_stream();
    if (!s)
        return FE_ENOMEM;
    s->n = n;
    s->T = T;
    s->prec = cfg->precision;
    s->fir_batches = 0;
    s->path = FE_PATH_AUTO;
    s->fft_parts = 0;
    s->Tk = s->prec == FE_PREC_FP32 ? kernel_taps(T) : kernel_taps_mfma(T);
    s->tap_scale = s->out_scale = 1.f;
    if (s->prec == FE_PREC_FP16) {
        // scale the taps so that the largest lies in [2^14, 2^15)
        float mx = 0.f;
        for (int64_t i = 0; i < int64_t(2) * n * T; ++i)
            mx = std::fmax(mx, std::fabs(cfg->weights[i]));
        if (!(mx < 3.0e38f)) {                 // inf or NaN taps
            delete s;
            return FE_EINVAL;
        }
        if (mx > 0.f) {
            const int sc = 14 - std::ilogb(mx);
            s->tap_scale = std::ldexp(1.f, sc);
            s->out_scale = std::ldexp(1.f, -sc);
        }
    }
    s->A = cfg->n_antennas;
    s->S = cfg->spectra_per_heap;
    s->D = cfg->max_delay;
    s->max_samples = cfg->max_samples;
    s->stream = static_cast<hipStream_t>(hip_stream);
    int64_t H = int64_t(2) * n * (s->Tk - 1) + s->D;
    H = (H + 15) / 16 * 16;                   // whole dwords of packed samples
    s->H = int(H);
    if (hipGetDevice(&s->device) != hipSuccess
        || hipDeviceGetAttribute(&s->cus, hipDeviceAttributeMultiprocessorCount, s->device) != hipSuccess) {
        delete s;
        return FE_EHIP;
    }
    s->cus = std::max(s->cus, 8);
    (void)scratch_address(s->device);       // set-up of fe_channelize_noalloc's scratch on this device

    const int streams = 2 * s->A;
    const int64_t n2 = 2 * int64_t(n);
    const size_t taps_n = size_t(n2) * s->Tk;
    const size_t hist_bytes = size_t(streams) * size_t(H * 5 / 4);
    const size_t g_floats = size_t(streams) * size_t(cfg->max_samples);
    std::vector<float2> tw = twiddles_for(n);
    std::vector<float2> tw16;
    std::vector<uint32_t> dfta;
    if (s->prec != FE_PREC_FP32 && n <= 8192) {
        tw16 = tw16_for(n);
        dfta = make_dft_a(s->prec);
    } else {
        tw16.assign(1, make_float2(0.f, 0.f));
        dfta.assign(4, 0u);
    }
    std::vector<float2> twf(1, make_float2(0.f, 0.f));
    if (n > 8192) {
        twf.resize(size_t(n));
        const long double pi = 3.141592653589793238462643383279503L;
        for (int gam = 0; gam < n / 16; ++gam)
            for (int d = 0; d < 16; ++d) {
                const long double a = -2.0L * pi * (long double)((int64_t(gam) * d) % n) / (long double)n;
                twf[size_t(gam) * 16 + d] = make_float2(float(std::cos(a)), float(std::sin(a)));
            }
    }
    bool ok = hipMalloc(&s->d_taps, taps_n * sizeof(float)) == hipSuccess
              && hipMalloc(&s->d_twf, twf.size() * sizeof(float2)) == hipSuccess
              && hipMalloc(&s->d_tw16, tw16.size() * sizeof(float2)) == hipSuccess
              && hipMalloc(&s->d_dfta, dfta.size() * sizeof(uint32_t)) == hipSuccess
              && hipMalloc(&s->d_tw, tw.size() * sizeof(float2)) == hipSuccess
              && hipMalloc(&s->d_untangle, size_t(n) * sizeof(float2)) == hipSuccess
              && (n <= 8192 || hipMalloc(&s->d_gpl, size_t(streams) * n * sizeof(float2)) == hipSuccess)
              && hipMalloc(&s->d_hist, hist_bytes) == hipSuccess
              && hipMalloc(&s->d_hist_tmp, hist_bytes) == hipSuccess
              && hipMalloc(&s->d_seam, size_t(seam_bytes(s))) == hipSuccess
              && hipMalloc(&s->d_g, g_floats * sizeof(float)) == hipSuccess
              && hipMalloc(&s->d_spec8, size_t(streams) * size_t(cfg->max_samples)) == hipSuccess
              && hipMalloc(&s->d_status, sizeof(int)) == hipSuccess;
    if (!ok) {
        free_stream(s);
        (void)hipGetLastError();
        return FE_ENOMEM;
    }

    std::vector<float> taps(taps_n, 0.f);
    std::memcpy(taps.data() + size_t(n2) * (s->Tk - T), cfg->weights, size_t(n2) * T * sizeof(float));
    std::vector<float2> unt(n);
    for (int k = 0; k < n; ++k) {
        const long double a = -3.141592653589793238462643383279503L * (long double)k / (long double)n;
        // the two-level FFT reads it in residue-plane order (channel d + 16 k' at d n/16 + k')
        const int pos = n > 8192 ? (k % 16) * (n / 16) + k / 16 : k;
        unt[pos] = make_float2(float(std::cos(a)), float(std::sin(a)));
    }
    ok = hipMemcpy(s->d_taps, taps.data(), taps_n * sizeof(float), hipMemcpyHostToDevice) == hipSuccess
         && hipMemcpy(s->d_tw, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice) == hipSuccess
         && hipMemcpy(s->d_untangle, unt.data(), size_t(n) * sizeof(float2), hipMemcpyHostToDevice) == hipSuccess
         && hipMemcpy(s->d_tw16, tw16.data(), tw16.size() * sizeof(float2), hipMemcpyHostToDevice) == hipSuccess
         && hipMemcpy(s->d_twf, twf.data(), twf.size() * sizeof(float2), hipMemcpyHostToDevice) == hipSuccess
         && hipMemcpy(s->d_dfta, dfta.data(), dfta.size() * sizeof(uint32_t), hipMemcpyHostToDevice) == hipSuccess
         && hipMemset(s->d_hist, 0, hist_bytes) == hipSuccess
         && hipMemset(s->d_hist_tmp, 0, hist_bytes) == hipSuccess
         && hipMemset(s->d_status, 0, sizeof(int)) == hipSuccess
         && hipDeviceSynchronize() == hipSuccess;
    if (!ok) {
        free_stream(s);
        return FE_EHIP;
    }
    *out = s;
    return FE_OK;
}

fe_status fe_stream_destroy(fe_stream *s)
{
    if (!s)
        return FE_OK;
    fe_status st = hip_status(hipStreamSynchronize(s->stream));
    free_stream(s);
    return st;
}

fe_status fe_stream_set_hip_stream(fe_stream *s, void *hip_stream)
{
    if (!s)
        return FE_EINVAL;
    s->stream = static_cast<hipStream_t>(hip_stream);
    return FE_OK;
}

fe_status fe_stream_reset(fe_stream *s)
{
    if (!s)
        return FE_EINVAL;
    const int64_t bytes = int64_t(2) * s->A * (int64_t(s->H) * 5 / 4);
    (void)hipGetLastError();
    hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(bytes, 256)), dim3(256), 0, s->stream,
                       s->d_hist, bytes, s->d_status);
    return hip_status(hipGetLastError());
}

fe_status fe_channelize(fe_stream *s, const uint8_t *raw, int64_t n_samples, const double *delays,
                        const double *phases, const float *gains, int8_t *out)
{
    if (!out)
        return FE_EINVAL;
    return channelize_impl(s, raw, n_samples, delays, phases, gains, out, nullptr, nullptr);
}

fe_status fe_channelize_noalloc(fe_stream *s, const uint8_t *raw, int64_t n_samples, const double *delays,
                                const double *phases, const float *gains, int8_t *out)
{
    if (!s || !out)
        return FE_EINVAL;
    uint8_t *base = scratch_address(s->device);
    if (!base)
        return FE_EHIP;
    return channelize_impl(s, raw, n_samples, delays, phases, gains, out, nullptr, nullptr, base);
}

fe_status fe_channelize_prequant(fe_stream *s, const uint8_t *raw, int64_t n_samples,
                                 const double *delays, const double *phases, const float *gains,
                                 float *y_out)
{
    if (!y_out)
        return FE_EINVAL;
    return channelize_impl(s, raw, n_samples, delays, phases, gains, nullptr, y_out, nullptr);
}

fe_status fe_channelize_fir(fe_stream *s, const uint8_t *raw, int64_t n_samples,
                            const double *delays, float *g_out)
{
    if (!g_out)
        return FE_EINVAL;
    return channelize_impl(s, raw, n_samples, delays, nullptr, nullptr, nullptr, nullptr, g_out);
}

fe_status fe_stream_status(fe_stream *s)
{
    if (!s)
        return FE_EINVAL;
    if (hipStreamSynchronize(s->stream) != hipSuccess)
        return FE_EHIP;
    int v = 0;
    if (hipMemcpy(&v, s->d_status, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return FE_EHIP;
    return v ? FE_EDELAY : FE_OK;
}

fe_status fe_stream_timing(fe_stream *s, int enable)
{
    if (!s)
        return FE_EINVAL;
    if (!enable) {
        if (hipStreamSynchronize(s->stream) != hipSuccess)
            return FE_EHIP;
        free_events(s);
        return FE_OK;
    }
    if (s->ev.empty()) {
        s->ev.assign(size_t(EV_PER_CALL) * 4096, nullptr);
        for (hipEvent_t &e : s->ev)
            if (hipEventCreate(&e) != hipSuccess) {
                free_events(s);
                return FE_EHIP;
            }
    }
    s->ev_used = 0;
    s->timing = true;
    return FE_OK;
}

fe_status fe_stream_timing_read(fe_stream *s, double *fir_ms, double *post_ms, double *turn_ms,
                                int64_t *calls)
{
    if (!s)
        return FE_EINVAL;
    double acc[3] = {0.0, 0.0, 0.0};
    if (s->ev_used > 0 && hipStreamSynchronize(s->stream) != hipSuccess)
        return FE_EHIP;
    for (int i = 0; i < s->ev_used; ++i) {
        hipEvent_t *e = &s->ev[size_t(i) * EV_PER_CALL];
        const int from[3] = {0, 2, 3}, to[3] = {1, 3, 4};
        for (int k = 0; k < 3; ++k) {
            float x = 0.f;
            if (hipEventElapsedTime(&x, e[from[k]], e[to[k]]) != hipSuccess)
                return FE_EHIP;
            acc[k] += x;
        }
    }
    if (fir_ms)
        *fir_ms = acc[0];
    if (post_ms)
        *post_ms = acc[1];
    if (turn_ms)
        *turn_ms = acc[2];
    if (calls)
        *calls = s->ev_used;
    s->ev_used = 0;
    return FE_OK;
}

fe_status fe_debug_unpack10(const uint8_t *raw, int64_t first, int64_t count, int32_t *out,
                            void *hip_stream)
{
    if (!raw || !out || first < 0 || count < 0)
        return FE_EINVAL;
    if (count == 0)
        return FE_OK;
    (void)hipGetLastError();
    hipLaunchKernelGGL(unpack_kernel, dim3(grid_for(count, 256)), dim3(256), 0,
                       static_cast<hipStream_t>(hip_stream), raw, first, count, out);
    return hip_status(hipGetLastError());
}

const char *fe_strerror(fe_status status)
{
    switch (status) {
    case FE_OK: return "success";
    case FE_EINVAL: return "invalid argument";
    case FE_ENOMEM: return "device allocation failed";
    case FE_EHIP: return "HIP runtime error";
    case FE_EDELAY: return "coarse delay outside [0, max_delay] (spectrum zeroed)";
    case FE_ESIZE: return "n_samples exceeds the stream's max_samples";
    default: return "unknown status";
    }
}

int32_t fe_version(void) { return 200; }

// ---------------------------------------------------------------------------
// Autotuning and batches
// ---------------------------------------------------------------------------

fe_status fe_stream_autotune(fe_stream *s, const uint8_t *raw, int64_t n_samples, const double *delays,
                             const double *phases, const float *gains, int8_t *out, int iters,
                             int *choice)
{
    if (!s || !out || iters < 1)
        return FE_EINVAL;
    fe_status st = check_call(s, raw, n_samples, delays);
    if (st != FE_OK)
        return st;
    if (!phases || !gains)
        return FE_EINVAL;
    // candidates: FIR runs of 1, 2, 4, 8 batches (FP32 FIR only), and the
    // per-launch choice; each timed with HIP events over `iters` calls
    // FIR run length in batches of spectra (FP32), or spectrum tiles per
    // workgroup chain (matrix-core FIR); 0 = the per-launch default
    // (fused path: workgroups per CU, same candidates), for each of the paths
    // the stream can run
    static const int cand[] = {0, 1, 2, 4, 8};
    const int ncand = 5;
    // (the FIR engine of FP16/BF16 streams is left as set: the two engines
    // round differently, and tuning keeps results bit for bit)
    int paths[3], npaths = 0;
    if (s->prec == FE_PREC_FP32) {
        paths[npaths++] = FE_PATH_SPLIT;
        if (s->n <= 8192)
            paths[npaths++] = FE_PATH_SPLIT_FOLDED;
        if (fused_eligible(s))
            paths[npaths++] = FE_PATH_FUSED;
    } else if (!matrix_fir(s)) {
        paths[npaths++] = FE_PATH_SPLIT;
        paths[npaths++] = FE_PATH_SPLIT_FOLDED;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0)
            (void)hipEventDestroy(e0);
        return FE_EHIP;
    }
    const int saved = s->fir_batches, saved_path = s->path;
    const bool timing = s->timing;
    s->timing = false;
    float best_ms = 3.0e38f;
    int best = 0, best_path = saved_path;
    st = FE_OK;
    for (int c = 0; c < ncand * std::max(npaths, 1) && st == FE_OK; ++c) {
        s->path = npaths > 0 ? paths[c / ncand] : saved_path;
        s->fir_batches = cand[c % ncand];
        st = channelize_impl(s, raw, n_samples, delays, phases, gains, out, nullptr, nullptr);   // warm
        if (st != FE_OK)
            break;
        (void)hipEventRecord(e0, s->stream);
        for (int i = 0; i < iters && st == FE_OK; ++i)
            st = channelize_impl(s, raw, n_samples, delays, phases, gains, out, nullptr, nullptr);
        (void)hipEventRecord(e1, s->stream);
        if (hipEventSynchronize(e1) != hipSuccess) {
            st = FE_EHIP;
            break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best_ms) {
            best_ms = ms;
            best = cand[c % ncand];
            best_path = s->path;
        }
    }
    s->fir_batches = st == FE_OK ? best : saved;
    s->path = st == FE_OK ? best_path : saved_path;
    // then, above 8192 channels, the post kernel's split of a spectrum's
    // rounds over workgroups (results are bit-identical for every split)
    if (st == FE_OK && s->n > 8192) {
        static const int parts[] = {0, 1, 3, 9};
        const int saved_parts = s->fft_parts;
        float best_p = 3.0e38f;
        int best_parts = saved_parts;
        for (int c = 0; c < 4 && st == FE_OK; ++c) {
            s->fft_parts = parts[c];
            st = channelize_impl(s, raw, n_samples, delays, phases, gains, out, nullptr, nullptr);   // warm
            if (st != FE_OK)
                break;
            (void)hipEventRecord(e0, s->stream);
            for (int i = 0; i < iters && st == FE_OK; ++i)
                st = channelize_impl(s, raw, n_samples, delays, phases, gains, out, nullptr, nullptr);
            (void)hipEventRecord(e1, s->stream);
            if (hipEventSynchronize(e1) != hipSuccess) {
                st = FE_EHIP;
                break;
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < best_p) {
                best_p = ms;
                best_parts = parts[c];
            }
        }
        s->fft_parts = st == FE_OK ? best_parts : saved_parts;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    s->timing = timing;
    if (choice)
        *choice = s->fir_batches;
    // the timing calls advanced the stream like real calls: restart it
    if (st == FE_OK)
        st = fe_stream_reset(s);
    return st;
}

fe_status fe_stream_set_fft_parts(fe_stream *s, int parts)
{
    if (!s || parts < 0 || parts > 9)
        return FE_EINVAL;
    s->fft_parts = parts;
    return FE_OK;
}

fe_status fe_stream_get_fft_parts(const fe_stream *s, int *parts)
{
    if (!s || !parts)
        return FE_EINVAL;
    *parts = s->fft_parts;
    return FE_OK;
}

fe_status fe_stream_set_tuning(fe_stream *s, int fir_batches)
{
    if (!s || fir_batches < 0 || fir_batches > 64)
        return FE_EINVAL;
    s->fir_batches = fir_batches;
    return FE_OK;
}

fe_status fe_stream_set_schedule(fe_stream *s, int path, int fir_batches)
{
    if (!s || fir_batches < 0 || fir_batches > 64
        || (path != FE_PATH_AUTO && path != FE_PATH_SPLIT && path != FE_PATH_FUSED
            && path != FE_PATH_MATRIX_FIR && path != FE_PATH_SPLIT_FOLDED))
        return FE_EINVAL;
    s->path = path;
    s->fir_batches = fir_batches;
    return FE_OK;
}

fe_status fe_stream_get_schedule(const fe_stream *s, int *path, int *fir_batches)
{
    if (!s)
        return FE_EINVAL;
    if (path)
        *path = fused_path(s) ? FE_PATH_FUSED : matrix_fir(s) ? FE_PATH_MATRIX_FIR
                : heap_fold(s, int(s->max_samples / (2 * s->n))) ? FE_PATH_SPLIT_FOLDED : FE_PATH_SPLIT;
    if (fir_batches)
        *fir_batches = s->fir_batches;
    return FE_OK;
}

}  // extern "C"

struct fe_batch {
    std::vector<fe_stream *> members;
    hipStream_t main;
    hipStream_t cap;                       // capture origin (the legacy default stream cannot be captured)
    std::vector<hipStream_t> forks;        // one per member, default priority
    std::vector<hipEvent_t> join;          // one per member
    hipEvent_t fork_ev;
    hipGraph_t graph;
    hipGraphExec_t exec;
    // job tables of the grouped launches: one for the captured graph, one for
    // eager runs (uploaded from pinned host memory on the batch stream)
    size_t jobs_cap;                       // bytes of each table
    uint8_t *d_jobs_graph;
    uint8_t *d_jobs_eager;
    uint8_t *h_jobs;
    hipEvent_t upload_ev;
    bool upload_pending;
    bool grouped;                          // grouped launches (else every member on its fork stream)
    hipStream_t gs[6];                     // grouped launches: one stream per FIR / FFT group
    hipEvent_t gev[6];
    hipEvent_t fir_done;
};

namespace {

void free_batch(fe_batch *b)
{
    if (!b)
        return;
    for (int k = 0; k < 6; ++k) {
        if (b->gs[k])
            (void)hipStreamDestroy(b->gs[k]);
        if (b->gev[k])
            (void)hipEventDestroy(b->gev[k]);
    }
    if (b->fir_done)
        (void)hipEventDestroy(b->fir_done);
    (void)hipFree(b->d_jobs_graph);
    (void)hipFree(b->d_jobs_eager);
    if (b->h_jobs)
        (void)hipHostFree(b->h_jobs);
    if (b->upload_ev)
        (void)hipEventDestroy(b->upload_ev);
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    for (hipEvent_t e : b->join)
        if (e)
            (void)hipEventDestroy(e);
    if (b->fork_ev)
        (void)hipEventDestroy(b->fork_ev);
    for (hipStream_t st : b->forks)
        if (st)
            (void)hipStreamDestroy(st);
    if (b->cap)
        (void)hipStreamDestroy(b->cap);
    delete b;
}

// Members run by the grouped launches: FP32 streams on the split path.
bool grouped_member(const fe_stream *s) { return s->prec == FE_PREC_FP32 && !fused_path(s); }

// Job tables of one batch step and the launches that read them (offsets into
// one byte table).
struct BatchPlan {
    std::vector<uint8_t> table;
    struct Launch {
        int kind;                          // 0 copy, 1 FIR (by taps), 2 FFT/post (by n), 3 turn
        int param;                         // taps or n
        size_t off;
        int count;
        int64_t units;                     // blocks (copy: words)
    };
    std::vector<Launch> pre, mid, post;    // before the FIR (seam staging), FIR + history, FFT/post + turn
    std::vector<int> short_calls;          // members whose call is shorter than their history
    std::vector<int> large;                // members with n > 8192 (their FFT runs per member)
};

template <typename J>
void plan_add(BatchPlan &P, std::vector<BatchPlan::Launch> &list, int kind, int param, const std::vector<J> &jobs,
              int64_t units)
{
    if (jobs.empty())
        return;
    size_t off = (P.table.size() + 63) / 64 * 64;
    P.table.resize(off + jobs.size() * sizeof(J));
    std::memcpy(P.table.data() + off, jobs.data(), jobs.size() * sizeof(J));
    list.push_back({kind, param, off, int(jobs.size()), units});
}

// FIR run length over `spectra` spectra (as launch_fir_range)
int fir_run_length(const fe_stream *s, int T, int spectra)
{
    const int streams = 2 * s->A, colblocks = 2 * s->n / (2 * FIR_THREADS), B = (64 / T) * T;
    if (s->fir_batches > 0)
        return s->fir_batches * B;
    int R = 4 * B;
    while (R > B && int64_t(streams) * ((spectra + R - 1) / R) * colblocks < 2048)
        R -= B;
    return R;
}

void build_plan(const fe_batch *b, const fe_call *calls, BatchPlan &P)
{
    std::vector<CopyJob> stage, hist;
    int64_t stage_w = 0, hist_w = 0;
    static const int taps_k[] = {4, 8, 16, 24, 32};
    static const int ns_k[] = {256, 512, 1024, 2048, 4096, 8192};
    std::vector<FirJob> fir[5];
    int64_t fir_b[5] = {0, 0, 0, 0, 0};
    std::vector<PostJob> post[6];
    int64_t post_b[6] = {0, 0, 0, 0, 0, 0};
    std::vector<TurnJob> turn;
    int64_t turn_b = 0;
    for (size_t i = 0; i < b->members.size(); ++i) {
        const fe_stream *s = b->members[i];
        if (!grouped_member(s))
            continue;
        const fe_call &c = calls[i];
        const int64_t N = c.n_samples;
        const int n2 = 2 * s->n, M = int(N / n2), streams = 2 * s->A, T = s->Tk;
        const int64_t row_bytes = int64_t(n2) * 5 / 4, hb = int64_t(s->H) * 5 / 4, nb = N * 5 / 4;
        const int ti = int(std::find(taps_k, taps_k + 5, T) - taps_k);
        FirJob F = {};
        F.hist = s->d_hist;
        F.hist_stride = hb;
        F.taps = s->d_taps;
        F.delays = c.delays;
        F.g = s->d_g;
        F.H = s->H;
        F.n2 = n2;
        F.M = M;
        F.D = s->D;
        F.colblocks = n2 / (2 * FIR_THREADS);
        // the seam from a staging buffer, the rest from the chunk
        const int S0 = std::min(M, seam_spectra(s)), K = seam_rows_before(s), rows = K + S0;
        CopyJob C = {};
        C.dst = reinterpret_cast<uint32_t *>(s->d_seam);
        C.dst_stride = rows * row_bytes / 4;
        C.src1 = reinterpret_cast<const uint32_t *>(s->d_hist);
        C.src1_stride = hb / 4;
        C.src2 = reinterpret_cast<const uint32_t *>(c.raw);
        C.src2_stride = nb / 4;
        C.z = (int64_t(K) * n2 - s->H) * 5 / 16;
        C.h = hb / 4;
        C.len = rows * row_bytes / 4;
        C.streams = streams;
        C.begin = stage_w;
        stage_w += C.len * streams;
        stage.push_back(C);
        F.raw = s->d_seam;
        F.raw_stride = rows * row_bytes;
        F.mb = K;
        F.me = K + S0;
        F.moff = K;
        F.mrows = rows;
        F.R = fir_run_length(s, T, S0);
        F.runs = (S0 + F.R - 1) / F.R;
        F.begin = int(fir_b[ti]);
        fir_b[ti] += int64_t(streams) * F.runs * F.colblocks;
        fir[ti].push_back(F);
        if (S0 < M) {
            F.raw = c.raw;
            F.raw_stride = nb;
            F.mb = S0;
            F.me = M;
            F.moff = 0;
            F.mrows = M;
            F.R = fir_run_length(s, T, M - S0);
            F.runs = (M - S0 + F.R - 1) / F.R;
            F.begin = int(fir_b[ti]);
            fir_b[ti] += int64_t(streams) * F.runs * F.colblocks;
            fir[ti].push_back(F);
        }
        // the history: the chunk's last H samples (shorter calls per member)
        if (N >= s->H) {
            CopyJob Hj = {};
            Hj.dst = reinterpret_cast<uint32_t *>(s->d_hist);
            Hj.dst_stride = hb / 4;
            Hj.src2 = reinterpret_cast<const uint32_t *>(c.raw);
            Hj.src2_stride = nb / 4;
            Hj.src2_off = (nb - hb) / 4;
            Hj.len = hb / 4;
            Hj.streams = streams;
            Hj.begin = hist_w;
            hist_w += Hj.len * streams;
            hist.push_back(Hj);
        } else {
            P.short_calls.push_back(int(i));
        }
        if (s->n > 8192) {
            P.large.push_back(int(i));
        } else {
            const int ni = int(std::find(ns_k, ns_k + 6, s->n) - ns_k);
            PostJob Q = {};
            Q.g = s->d_g;
            Q.delays = c.delays;
            Q.phases = c.phases;
            Q.gains = reinterpret_cast<const float2 *>(c.gains);
            Q.tw = s->d_tw;
            Q.untangle = s->d_untangle;
            Q.spec8 = s->d_spec8;
            Q.status = s->d_status;
            Q.M = M;
            Q.D = s->D;
            Q.begin = int(post_b[ni]);
            post_b[ni] += int64_t(s->A) * M * 2;
            post[ni].push_back(Q);
        }
        TurnJob U = {};
        U.spec8 = s->d_spec8;
        U.out = c.out;
        U.M = M;
        U.n = s->n;
        U.S = s->S;
        U.ftiles = (M + CT - 1) / CT;
        U.ktiles = s->n / CT;
        U.ns = s->n > 8192 ? s->n / 16 : 0;
        U.begin = int(turn_b);
        turn_b += int64_t(s->A) * U.ftiles * U.ktiles;
        turn.push_back(U);
    }
    plan_add(P, P.pre, 0, 0, stage, stage_w);
    for (int t = 0; t < 5; ++t)
        plan_add(P, P.mid, 1, taps_k[t], fir[t], fir_b[t]);
    plan_add(P, P.mid, 0, 0, hist, hist_w);
    for (int k = 0; k < 6; ++k)
        plan_add(P, P.post, 2, ns_k[k], post[k], post_b[k]);
    plan_add(P, P.post, 3, 0, turn, turn_b);
}

void launch_plan_list(const std::vector<BatchPlan::Launch> &list, const uint8_t *table, hipStream_t st)
{
    for (const BatchPlan::Launch &L : list) {
        const void *j = table + L.off;
        const unsigned blocks = unsigned(L.units);
        switch (L.kind) {
        case 0:
            hipLaunchKernelGGL(copy_jobs_kernel, dim3(grid_for(L.units, 256)), dim3(256), 0, st,
                               static_cast<const CopyJob *>(j), L.count, L.units);
            break;
        case 1: {
            const FirJob *f = static_cast<const FirJob *>(j);
            switch (L.param) {
            case 4: hipLaunchKernelGGL((fir_jobs_kernel<4>), dim3(blocks), dim3(FIR_THREADS), 0, st, f, L.count); break;
            case 8: hipLaunchKernelGGL((fir_jobs_kernel<8>), dim3(blocks), dim3(FIR_THREADS), 0, st, f, L.count); break;
            case 16: hipLaunchKernelGGL((fir_jobs_kernel<16>), dim3(blocks), dim3(FIR_THREADS), 0, st, f, L.count); break;
            case 24: hipLaunchKernelGGL((fir_jobs_kernel<24>), dim3(blocks), dim3(FIR_THREADS), 0, st, f, L.count); break;
            case 32: hipLaunchKernelGGL((fir_jobs_kernel<32>), dim3(blocks), dim3(FIR_THREADS), 0, st, f, L.count); break;
            }
            break;
        }
        case 2: {
            const PostJob *q = static_cast<const PostJob *>(j);
            switch (L.param) {
            case 256: hipLaunchKernelGGL((post_jobs_kernel<256>), dim3(blocks), dim3(256 / 16), 0, st, q, L.count); break;
            case 512: hipLaunchKernelGGL((post_jobs_kernel<512>), dim3(blocks), dim3(512 / 16), 0, st, q, L.count); break;
            case 1024: hipLaunchKernelGGL((post_jobs_kernel<1024>), dim3(blocks), dim3(1024 / 16), 0, st, q, L.count); break;
            case 2048: hipLaunchKernelGGL((post_jobs_kernel<2048>), dim3(blocks), dim3(2048 / 16), 0, st, q, L.count); break;
            case 4096: hipLaunchKernelGGL((post_jobs_kernel<4096>), dim3(blocks), dim3(4096 / 16), 0, st, q, L.count); break;
            case 8192: hipLaunchKernelGGL((post_jobs_kernel<8192>), dim3(blocks), dim3(8192 / 16), 0, st, q, L.count); break;
            }
            break;
        }
        case 3:
            hipLaunchKernelGGL(turn_jobs_kernel, dim3(blocks), dim3(256), 0, st, static_cast<const TurnJob *>(j),
                               L.count);
            break;
        }
    }
}

// Enqueue one step: the members outside the grouped launches (fused-path and
// matrix-core streams) each on a fork stream of their own; the FP32 split
// members through the grouped launches on the origin stream (job table
// `table`, device, already holding plan P's jobs); then the origin stream
// waits for the forks.
fe_status batch_enqueue_grouped(fe_batch *b, const fe_call *calls, hipStream_t origin, const BatchPlan &P,
                                const uint8_t *table)
{
    if (hipEventRecord(b->fork_ev, origin) != hipSuccess)
        return FE_EHIP;
    fe_status st = FE_OK;
    std::vector<size_t> forked;
    for (size_t i = 0; i < b->members.size() && st == FE_OK; ++i) {
        fe_stream *m = b->members[i];
        if (grouped_member(m))
            continue;
        const fe_call &c = calls[i];
        if (hipStreamWaitEvent(b->forks[i], b->fork_ev, 0) != hipSuccess)
            return FE_EHIP;
        hipStream_t saved = m->stream;
        const bool timing = m->timing;
        m->stream = b->forks[i];
        m->timing = false;
        st = channelize_impl(m, c.raw, c.n_samples, c.delays, c.phases, c.gains, c.out, nullptr, nullptr);
        m->stream = saved;
        m->timing = timing;
        if (st == FE_OK && hipEventRecord(b->join[i], b->forks[i]) != hipSuccess)
            st = FE_EHIP;
        forked.push_back(i);
    }
    if (st == FE_OK) {
        // seam staging on the origin stream; then each FIR group (one per
        // tap count) on a group stream of its own; once all have finished,
        // the history copies on the origin stream beside each FFT group (one
        // per channel count) and each large-n member's two-level FFT on
        // streams of their own; the corner turn after all of them
        (void)hipGetLastError();
        launch_plan_list(P.pre, table, origin);
        bool ok = hipEventRecord(b->fir_done, origin) == hipSuccess;
        std::vector<BatchPlan::Launch> firs, hists, posts, turns;
        for (const BatchPlan::Launch &L : P.mid)
            (L.kind == 1 ? firs : hists).push_back(L);
        for (const BatchPlan::Launch &L : P.post)
            (L.kind == 2 ? posts : turns).push_back(L);
        for (size_t k = 0; k < firs.size() && ok; ++k) {
            ok = hipStreamWaitEvent(b->gs[k], b->fir_done, 0) == hipSuccess;
            launch_plan_list(std::vector<BatchPlan::Launch>(1, firs[k]), table, b->gs[k]);
            ok = ok && hipEventRecord(b->gev[k], b->gs[k]) == hipSuccess
                 && hipStreamWaitEvent(origin, b->gev[k], 0) == hipSuccess;
        }
        ok = ok && hipEventRecord(b->fir_done, origin) == hipSuccess;
        for (size_t k = 0; k < posts.size() && ok; ++k) {
            ok = hipStreamWaitEvent(b->gs[k], b->fir_done, 0) == hipSuccess;
            launch_plan_list(std::vector<BatchPlan::Launch>(1, posts[k]), table, b->gs[k]);
            ok = ok && hipEventRecord(b->gev[k], b->gs[k]) == hipSuccess;
        }
        for (int i : P.large) {
            if (!ok)
                break;
            fe_stream *m = b->members[size_t(i)];
            const fe_call &c = calls[i];
            const Work wk = {m->d_g, m->d_spec8, m->d_gpl, m->d_hist_tmp, m->d_seam};
            const int M = int(c.n_samples / (2 * m->n));
            ok = hipStreamWaitEvent(b->forks[size_t(i)], b->fir_done, 0) == hipSuccess;
            hipStream_t saved = m->stream;
            m->stream = b->forks[size_t(i)];
            launch_post(m, wk, M, c.delays, c.phases, c.gains, nullptr, 0, M);
            m->stream = saved;
            ok = ok && hipEventRecord(b->join[size_t(i)], b->forks[size_t(i)]) == hipSuccess;
        }
        launch_plan_list(hists, table, origin);
        for (int i : P.short_calls) {
            fe_stream *m = b->members[size_t(i)];
            const Work wk = {m->d_g, m->d_spec8, m->d_gpl, m->d_hist_tmp, m->d_seam};
            hipStream_t saved = m->stream;
            m->stream = origin;
            launch_history_update(m, wk, calls[i].raw, calls[i].n_samples);
            m->stream = saved;
        }
        for (size_t k = 0; k < posts.size() && ok; ++k)
            ok = hipStreamWaitEvent(origin, b->gev[k], 0) == hipSuccess;
        for (int i : P.large)
            ok = ok && hipStreamWaitEvent(origin, b->join[size_t(i)], 0) == hipSuccess;
        launch_plan_list(turns, table, origin);
        st = ok ? hip_status(hipGetLastError()) : FE_EHIP;
    }
    for (size_t i : forked)
        if (hipStreamWaitEvent(origin, b->join[i], 0) != hipSuccess && st == FE_OK)
            st = FE_EHIP;
    return st;
}

// Enqueue every member's call: the fork streams wait for the batch stream,
// each member runs on its own fork stream, the batch stream waits for all.
fe_status batch_enqueue(fe_batch *b, const fe_call *calls, hipStream_t origin)
{
    if (hipEventRecord(b->fork_ev, origin) != hipSuccess)
        return FE_EHIP;
    fe_status st = FE_OK;
    for (size_t i = 0; i < b->members.size() && st == FE_OK; ++i) {
        fe_stream *m = b->members[i];
        const fe_call &c = calls[i];
        if (hipStreamWaitEvent(b->forks[i], b->fork_ev, 0) != hipSuccess)
            return FE_EHIP;
        hipStream_t saved = m->stream;
        const bool timing = m->timing;
        m->stream = b->forks[i];
        m->timing = false;
        st = c.out ? channelize_impl(m, c.raw, c.n_samples, c.delays, c.phases, c.gains, c.out, nullptr, nullptr)
                   : FE_EINVAL;
        m->stream = saved;
        m->timing = timing;
        if (st == FE_OK && hipEventRecord(b->join[i], b->forks[i]) != hipSuccess)
            st = FE_EHIP;
    }
    for (size_t i = 0; i < b->members.size(); ++i)
        if (hipStreamWaitEvent(origin, b->join[i], 0) != hipSuccess && st == FE_OK)
            st = FE_EHIP;
    return st;
}

fe_status batch_check(const fe_batch *b, const fe_call *calls)
{
    if (!b || !calls)
        return FE_EINVAL;
    for (size_t i = 0; i < b->members.size(); ++i) {
        const fe_call &c = calls[i];
        fe_status st = check_call(b->members[i], c.raw, c.n_samples, c.delays);
        if (st != FE_OK)
            return st;
        if (!c.phases || !c.gains || !c.out)
            return FE_EINVAL;
    }
    return FE_OK;
}

}  // namespace

extern "C" {

fe_status fe_batch_create(fe_stream *const *members, int count, void *hip_stream, fe_batch **out)
{
    if (!members || count < 1 || !out)
        return FE_EINVAL;
    for (int i = 0; i < count; ++i)
        if (!members[i])
            return FE_EINVAL;
    fe_batch *b = new (std::nothrow) fe_batch();
    if (!b)
        return FE_ENOMEM;
    b->members.assign(members, members + count);
    b->main = static_cast<hipStream_t>(hip_stream);
    b->forks.assign(size_t(count), nullptr);
    b->join.assign(size_t(count), nullptr);
    b->fork_ev = nullptr;
    b->graph = nullptr;
    b->exec = nullptr;
    b->cap = nullptr;
    b->d_jobs_graph = b->d_jobs_eager = b->h_jobs = nullptr;
    b->upload_ev = nullptr;
    b->upload_pending = false;
    b->grouped = false;                    // per-member fork streams measure faster
    for (int k = 0; k < 6; ++k) {
        b->gs[k] = nullptr;
        b->gev[k] = nullptr;
    }
    b->fir_done = nullptr;
    b->jobs_cap = size_t(count) * (2 * sizeof(FirJob) + sizeof(PostJob) + sizeof(TurnJob) + 2 * sizeof(CopyJob))
                  + 64 * 16;
    bool ok = hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming) == hipSuccess
              && hipEventCreateWithFlags(&b->upload_ev, hipEventDisableTiming) == hipSuccess
              && hipMalloc(&b->d_jobs_graph, b->jobs_cap) == hipSuccess
              && hipMalloc(&b->d_jobs_eager, b->jobs_cap) == hipSuccess
              && hipHostMalloc(&b->h_jobs, b->jobs_cap, hipHostMallocDefault) == hipSuccess
              && hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) == hipSuccess
              && hipEventCreateWithFlags(&b->fir_done, hipEventDisableTiming) == hipSuccess;
    for (int k = 0; k < 6 && ok; ++k)
        ok = hipStreamCreateWithFlags(&b->gs[k], hipStreamNonBlocking) == hipSuccess
             && hipEventCreateWithFlags(&b->gev[k], hipEventDisableTiming) == hipSuccess;
    for (int i = 0; i < count && ok; ++i)
        ok = hipStreamCreateWithFlags(&b->forks[size_t(i)], hipStreamNonBlocking) == hipSuccess
             && hipEventCreateWithFlags(&b->join[size_t(i)], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        free_batch(b);
        return FE_EHIP;
    }
    *out = b;
    return FE_OK;
}

fe_status fe_batch_destroy(fe_batch *b)
{
    if (!b)
        return FE_OK;
    fe_status st = hip_status(hipStreamSynchronize(b->main));
    if (b->cap && hipStreamSynchronize(b->cap) != hipSuccess)
        st = FE_EHIP;
    for (hipStream_t f : b->forks)
        if (f && hipStreamSynchronize(f) != hipSuccess)
            st = FE_EHIP;
    for (hipStream_t f : b->gs)
        if (f && hipStreamSynchronize(f) != hipSuccess)
            st = FE_EHIP;
    free_batch(b);
    return st;
}

fe_status fe_batch_run(fe_batch *b, const fe_call *calls)
{
    fe_status st = batch_check(b, calls);
    if (st != FE_OK)
        return st;
    if (!b->grouped)
        return batch_enqueue(b, calls, b->main);
    BatchPlan P;
    build_plan(b, calls, P);
    if (P.table.size() > b->jobs_cap)
        return FE_EINVAL;
    // the pinned staging is rewritten once its last upload has been read
    if (b->upload_pending && hipEventSynchronize(b->upload_ev) != hipSuccess)
        return FE_EHIP;
    if (!P.table.empty()) {
        std::memcpy(b->h_jobs, P.table.data(), P.table.size());
        if (hipMemcpyAsync(b->d_jobs_eager, b->h_jobs, P.table.size(), hipMemcpyHostToDevice, b->main) != hipSuccess
            || hipEventRecord(b->upload_ev, b->main) != hipSuccess)
            return FE_EHIP;
        b->upload_pending = true;
    }
    return batch_enqueue_grouped(b, calls, b->main, P, b->d_jobs_eager);
}

fe_status fe_batch_set_grouped(fe_batch *b, int grouped)
{
    if (!b)
        return FE_EINVAL;
    b->grouped = grouped != 0;
    return FE_OK;
}

fe_status fe_batch_capture(fe_batch *b, const fe_call *calls)
{
    fe_status st = batch_check(b, calls);
    if (st != FE_OK)
        return st;
    if (hipStreamSynchronize(b->main) != hipSuccess)
        return FE_EHIP;
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    BatchPlan P;
    if (b->grouped) {
        // the graph's job table is written once, before the capture
        build_plan(b, calls, P);
        if (P.table.size() > b->jobs_cap)
            return FE_EINVAL;
        if (!P.table.empty()
            && hipMemcpy(b->d_jobs_graph, P.table.data(), P.table.size(), hipMemcpyHostToDevice) != hipSuccess)
            return FE_EHIP;
    }
    if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return FE_EHIP;
    st = b->grouped ? batch_enqueue_grouped(b, calls, b->cap, P, b->d_jobs_graph) : batch_enqueue(b, calls, b->cap);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(b->cap, &g);
    if (st != FE_OK || ec != hipSuccess || !g) {
        if (g)
            (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return st != FE_OK ? st : FE_EHIP;
    }
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        b->exec = nullptr;
        return FE_EHIP;
    }
    return FE_OK;
}

fe_status fe_batch_launch(fe_batch *b)
{
    if (!b || !b->exec)
        return FE_EINVAL;
    return hip_status(hipGraphLaunch(b->exec, b->main));
}

}  // extern "C"
