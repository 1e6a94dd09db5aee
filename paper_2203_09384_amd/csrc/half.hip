// FP16 / BF16 storage path, N = 2048: block floating point, every pass as
// dense DFT-matrix products on MFMA.
//
// The paper's library is FP32-only (section "Implementation"); this path
// stores data as half-precision (re, im) pairs and computes the same DFT of
// Eq. (dft) with the Cooley-Tukey split 2048 = 8 * 16 * 16:
//   pass A  radix 8 (NS = 1, no twiddles)
//   pass B  radix 16 (NS = 8)
//   pass C  radix 16 (NS = 128)
// Each pass is Y = F X for 16 butterflies at a time, F the DFT matrix of the
// radix, complex products written in real form with FP32 accumulation:
//   pass A  one v_mfma_f32_16x16x16_f16 per 16 butterflies: (re, im)
//           interleaved along both dimensions, so the stored (re, im) word
//           pairs are the data operand as they are;
//   passes B, C  two v_mfma_f32_16x16x32_f16 per 16 butterflies,
//           Re Y = [Re F | -Im F] [Re X; Im X],  Im Y = [Im F | Re F] [Re X; Im X].
// The inter-pass twiddles (FP32, from the plan's table) are folded into
// pass B's DFT operands or applied when pass B writes its outputs to LDS,
// so every data operand is a plain gather.
//
// Block floating point: logical value = stored * 2^exp[b] per transform.
// The input is scaled by a power of two so its largest component lies in
// [8, 16); with the at most 8 * 16 * 16 = 2^11 growth of the three passes
// no operand can exceed 2^15 < 65504, and the output is stored at that
// scale with exponent in_exp + e_max - 4 (- 11 for the inverse's 1/N,
// exact).  Scaling is by powers of two only, so it adds no rounding beyond
// the operands' own.
//
// MFMA operands are FP16 for both storage types.  After the block scaling
// every operand lies in FP16's range, FP16 carries three more significand
// bits than BF16 (a BF16 value converts to FP16 exactly), and the error of
// BF16 storage is set by the rounding of its output to BF16 (7 bits): FP16
// operands give the same error as BF16 operands split hi + lo (modelled
// 1.75e-3 against 1.72e-3) at one MFMA per product instead of three.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "device_fft.hpp"
#include "launch.hpp"
#include "half.hpp"

namespace mifft {
namespace {

typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef _Float16 v4h __attribute__((ext_vector_type(4)));
typedef _Float16 v2h __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef uint32_t v2u __attribute__((ext_vector_type(2)));

constexpr int HN = 2048;
constexpr int HWG = 256;

// LDS layouts, one per exchange, each conflict-free for both its writer and
// its reader (modelled on the 64 banks) and affine in the per-instruction
// indices, so every access is a per-thread base plus an immediate offset.
// Element d is one 32-bit word holding its (re, im) as two FP16 halves (the
// MFMA operand type, so rounding there is the operands' own rounding).
//   A -> B      : d + (d >> 3) + 16 (d >> 10)
//   B -> C      : d + (d >> 6)
// Pass C's results go out through a wavefront-private part of the A -> B
// buffer (see half_transform).
__device__ __forceinline__ int fA(int d) { return d + (d >> 3) + 16 * (d >> 10); }
__device__ __forceinline__ int fB(int d) { return d + (d >> 6); }
constexpr int BUFA = 2336;  // words of the A -> B buffer (fA(2047) + 1 = 2319, rounded up)
constexpr int BUFB = 2080;  // words of the B -> C buffer (fB(2047) + 1 = 2079, rounded up)
// store staging: wave w's 16 rows of 32 words at 584 w + 36 row, inside the
// words its own pass-A writes use plus padding no wave writes
constexpr int STAGE_WAVE = 584, STAGE_ROW = 36;

// ---- conversions (round to nearest even)
template <bool BF>
__device__ __forceinline__ float to_f32(uint16_t h)
{
    if constexpr (BF)
        return __builtin_bit_cast(float, (uint32_t)h << 16);
    else
        return (float)__builtin_bit_cast(_Float16, h);
}

// MFMA operand: 8 FP16 values.
struct Op8 {
    v8h hi;
    __device__ __forceinline__ void set(int i, float x) { hi[i] = (_Float16)x; }
};

__device__ __forceinline__ v4f mfma(const Op8& a, const Op8& b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a.hi, b.hi, c, 0, 0, 0);
}

template <int S>
__device__ __forceinline__ cf tw_at(const cf* __restrict__ tw, int idx)
{
    cf w = tw[idx];
    if constexpr (S > 0)
        w.y = -w.y;
    return w;
}

// This lane's rows of the A operands of the 16-point DFT with the twiddles
// of a Stockham pass folded in: A[m][r] = exp(S 2 pi i r (8 m + g) / 128),
// i.e. F[m][r] w_128^{g r} (g = 0: the plain DFT).  Real form over K = 32:
// A_re[m] = [Re A[m][.] | -Im A[m][.]], A_im[m] = [Im A[m][.] | Re A[m][.]];
// lane l holds row m = l % 16, columns k = 8 (l / 16) + i.  Entries are
// single lookups of the FP32 table w_2048^{16 e}, rounded once to FP16.
template <int S>
__device__ __forceinline__ void dft16_operands(Op8& are, Op8& aim, int lane, int g, const cf* __restrict__ tw)
{
    const int m = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        const int r = (kq & 1) * 8 + i;
        const int e = (r * (8 * m + g)) & 127;
        const cf z = tw[16 * e];
        const float c = z.x, sn = (float)(-S) * z.y;  // exp(S 2 pi i e / 128)
        if (kq < 2) {
            are.set(i, c);
            aim.set(i, sn);
        } else {
            are.set(i, -sn);
            aim.set(i, c);
        }
    }
}

// This lane's part of pass A's operand: the 8-point DFT F[m][r] =
// exp(S 2 pi i m r / 8) in real form with (re, im) interleaved along both
// dimensions, a 16 x 16 matrix over row 2m + c' (c' = 0: Re y_m, 1: Im y_m)
// and column 2r + c (c = 0: Re x_r, 1: Im x_r):
//   [Re F, -Im F]
//   [Im F,  Re F]   at rows 2m, 2m + 1 and columns 2r, 2r + 1.
// For v_mfma_f32_16x16x16_f16 lane l holds row l % 16, columns 4 (l / 16) + i.
// Entries are lookups of the FP32 table (w_2048^{256 e} = w_8^e), rounded
// once to FP16 (0, +-1 exact; +-sqrt(2)/2 to 2^-12 relative).
template <int S>
__device__ __forceinline__ v4h dft8_operand(int lane, const cf* __restrict__ tw)
{
    const int row = lane & 15, m = row >> 1, cp = row & 1, kq = lane >> 4;
    v4h a;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const int k = 4 * kq + i, r = k >> 1, cc = k & 1;
        const cf z = tw_at<S>(tw, 256 * ((m * r) & 7));
        const float v = cp == 0 ? (cc == 0 ? z.x : -z.y) : (cc == 0 ? z.y : z.x);
        a[i] = (_Float16)v;
    }
    return a;
}

// Per-thread constants of the kernel: MFMA operands, twiddles, offsets.
struct HalfCtx {
    v4h f8;                // pass A, the 8-point DFT
    Op8 a_re[2], a_im[2];  // pass B, group g = 2 wave + gg, twiddles folded
    Op8 f_re, f_im;        // pass C, plain DFT
    cf twBase[2], twStep;  // pass C twiddles of pass B output (gg, i): twBase[gg] twStep^i
    int oLd;               // word of this lane's first input load
    // LDS offsets: pass A writes (q = 0, first word; q adds 144, the second
    // word is the next), pass B reads / writes and pass C reads of gg = 0
    // (gg = 1 is 1, 1 and 16 words further: the layouts are affine there)
    int oWA, oRB, oWB, oRC;
    int oStW, oStR, oSt;   // store staging: write and read offsets, output element
    uint32_t sel;          // byte selector of this lane's halves (re: low, im: high)
    int tid, lane, wave;
};

// Two floats to one word of two halves (a low, b high), each rounded to
// nearest even: one packed convert (v_cvt_pk_f16_f32 / v_cvt_pk_bf16_f32).
typedef float v2f32 __attribute__((ext_vector_type(2)));
typedef __bf16 v2bf16 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pack_f16(float a, float b)
{
    const v2f32 f = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, v2h));
}

template <bool BF>
__device__ __forceinline__ uint32_t pack_store(float a, float b)
{
    const v2f32 f = {a, b};
    if constexpr (BF)
        return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, v2bf16));
    else
        return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, v2h));
}

// An MFMA operand from 8 packed words: this lane's half (re or im) of each.
__device__ __forceinline__ Op8 gather_op(const uint32_t (&w)[8], uint32_t sel)
{
    v4u q;
#pragma unroll
    for (int j = 0; j < 4; j++)
        q[j] = __builtin_amdgcn_perm(w[2 * j + 1], w[2 * j], sel);
    Op8 o;
    o.hi = __builtin_bit_cast(v8h, q);
    return o;
}

// Maximum over the wavefront of a non-negative float, in every lane.
// Non-negative floats order like their bit patterns, so the reduction runs
// on integers with DPP row shifts (a prefix maximum within each row of 16
// lanes), then row broadcasts 15 and 31, leaving the maximum in lane 63.
// Lanes without a DPP source read 0, the identity here.
__device__ __forceinline__ float wave_max_nonneg(float x)
{
    int v = __builtin_bit_cast(int, x);
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false));  // row_shr:1
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false));  // row_shr:2
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false));  // row_shr:4
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false));  // row_shr:8
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false));  // row_bcast:15 -> rows 1, 3
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false));  // row_bcast:31 -> rows 2, 3
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(v, 63));
}

// This lane's pass-A input words of transform b: for group q (butterflies
// j = 64 wave + 16 q + n, n = lane % 16) the inputs r = 2 kq and 2 kq + 1
// (kq = lane / 16) of butterfly j, x[j + 256 r], as u[2 q] and u[2 q + 1].
// Plain loads: for this pattern (runs of 64 bytes per instruction, the rest
// of each line read by the same wave's next instructions) nontemporal loads
// measured 15% slower, as did a plain copy of it (92 against 79 us at 512 MiB).
__device__ __forceinline__ void load_raw(uint32_t (&u)[8], const uint32_t* __restrict__ in, int64_t b, int off)
{
    const uint32_t* src = in + b * HN + off;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        u[2 * q] = src[16 * q];
        u[2 * q + 1] = src[16 * q + 256];
    }
}

// Largest magnitude among the 16 half-precision components held in 8 raw
// words, as a float.  Magnitudes of one 16-bit float format order like their
// bit patterns with the sign cleared, so this is an unsigned 16-bit maximum
// of the stored bits (two components per v_pk_max_u16); inf and NaN compare
// above every finite value.
typedef uint16_t v2u16 __attribute__((ext_vector_type(2)));
template <bool BF>
__device__ __forceinline__ float raw_absmax(const uint32_t (&u)[8])
{
    v2u16 m = __builtin_bit_cast(v2u16, u[0] & 0x7fff7fffu);
#pragma unroll
    for (int k = 1; k < 8; k++)
        m = __builtin_elementwise_max(m, __builtin_bit_cast(v2u16, u[k] & 0x7fff7fffu));
    return to_f32<BF>(m[0] > m[1] ? m[0] : m[1]);
}

// The wave's largest input magnitude of the transform in `u`, published in
// red[wave] for the block maximum.
template <bool BF>
__device__ __forceinline__ void publish_max(const HalfCtx& c, const uint32_t (&u)[8], float* red)
{
    const float mx = wave_max_nonneg(raw_absmax<BF>(u));
    if (c.lane == 0)
        red[c.wave] = mx;
}

// Block maximum (over the four waves' maxima) -> the power-of-two exponent
// e_max with max < 2^e_max (0 for an all-zero or non-finite transform).
__device__ __forceinline__ int block_exponent(const float* red)
{
    const float mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    int e_max = 0;
    if (mx > 0.f && mx <= 3.4e38f)
        (void)frexpf(mx, &e_max);
    return e_max;
}

// The raw words scaled by 2^sh (largest component into [8, 16)) as FP16
// (re, im) pairs: pass A's data operand.  Exact, or one rounding to nearest
// even where a value lands below FP16's normal range.  FP16 storage: packed
// FP16 multiplies by 2^sh (sh is uniform; two steps above 2^15, where the
// scale itself is not an FP16 value and every value grows, exactly).  BF16
// storage: widened to FP32, ldexp (exact, and no 2^sh factor that could
// overflow), one packed convert.
template <bool BF>
__device__ __forceinline__ void scale_operands(const uint32_t (&u)[8], uint32_t (&o)[8], int sh)
{
    if constexpr (BF) {
#pragma unroll
        for (int k = 0; k < 8; k++)
            o[k] = pack_f16(ldexpf(__builtin_bit_cast(float, u[k] << 16), sh),
                            ldexpf(__builtin_bit_cast(float, u[k] & 0xffff0000u), sh));
    } else {
        const int s1 = sh > 15 ? 15 : sh;
        const _Float16 f1 = (_Float16)ldexpf(1.0f, s1);
        const v2h m1 = {f1, f1};
#pragma unroll
        for (int k = 0; k < 8; k++)
            o[k] = __builtin_bit_cast(uint32_t, __builtin_bit_cast(v2h, u[k]) * m1);
        if (sh > 15) {
            const _Float16 f2 = (_Float16)ldexpf(1.0f, sh - 15);
            const v2h m2 = {f2, f2};
#pragma unroll
            for (int k = 0; k < 8; k++)
                o[k] = __builtin_bit_cast(uint32_t, __builtin_bit_cast(v2h, o[k]) * m2);
        }
    }
}

// An empty asm that takes `o` as read and rewritten: the values are
// computed where it stands and later code sees new values (nothing that
// produced them is moved past it, and their loads carry no later wait).
__device__ __forceinline__ void pin(uint32_t (&o)[8])
{
#pragma unroll
    for (int k = 0; k < 8; k++)
        asm volatile("" : "+v"(o[k]));
}

// One transform.  `op` holds its pass-A operand words (scaled, FP16; made
// by the previous transform, or before the loop) and e_max its block
// exponent; its raw words in `cur` are dead, so `cur` is refilled with
// transform `refill` right away and two transforms' loads stay in flight.
// `nxt` holds the next transform's raw words: after pass B its per-wave
// maxima go to `red`, and after the second barrier (when every wave's are
// there) its exponent and operand words are made for the next call.  Made at
// the start of a transform instead, the compiler's loop-wide count of
// outstanding memory operations waited there for the loads of the
// transform after it, issued only one transform earlier.
// X holds the A -> B exchange (and pass C's store staging), Y the B -> C
// exchange.  Two barriers per transform:
//  - X is written after the barrier that follows the previous transform's
//    reads of X (its second: pass B reads, and staging reads are the same
//    wave's own words), Y after the barrier that follows the previous
//    transform's reads of Y (this transform's first), so one buffer of each
//    serves every transform;
//  - `red` is written before this transform's second barrier and read
//    after it; the next write is in the next transform, after its first
//    barrier, which every wave reaches only after its read.
template <int S, bool BF>
__device__ __forceinline__ void half_transform(const HalfCtx& c, uint32_t (&op)[8], int& e_max, uint32_t (&cur)[8],
                                               const uint32_t (&nxt)[8], uint32_t* X, uint32_t* Y, float* red,
                                               const uint32_t* __restrict__ in, const int32_t* __restrict__ in_exp,
                                               uint32_t* __restrict__ out, int32_t* __restrict__ out_exp,
                                               int64_t b, int64_t refill, int64_t batch, int scale_log2)
{
    // This transform's input exponent is read before the refill is issued,
    // and the refill itself is unconditional (past the end of the batch it
    // re-reads the last transform, which every workgroup shares through
    // the cache): a load issued after the refill, or a refill under a
    // condition, would make the wait for `nxt` below cover the refill too.
    const int e_in = in_exp ? in_exp[b] : 0;
    load_raw(cur, in, refill < batch ? refill : batch - 1, c.oLd);
    const int e_out = e_in + e_max - 4 + scale_log2;

    // ---- pass A: radix 8 on MFMA, 16 butterflies j = 64 wave + 16 q + n per
    // product; outputs y_{2 kq}, y_{2 kq + 1} of butterfly j (this lane's
    // accumulators) to the Stockham positions d = 8 j + 2 kq, + 1
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const v2u w = {op[2 * q], op[2 * q + 1]};
        const v4f z = {0.f, 0.f, 0.f, 0.f};
        const v4f y = __builtin_amdgcn_mfma_f32_16x16x16f16(c.f8, __builtin_bit_cast(v4h, w), z, 0, 0, 0);
        uint32_t* wa = X + c.oWA + 144 * q;
        wa[0] = pack_f16(y[0], y[1]);
        wa[1] = pack_f16(y[2], y[3]);
    }
    __syncthreads();

    // ---- pass B: radix 16 (NS = 8) on MFMA.  Group g holds the 16 butterflies
    // j = g + 8 n (all with j mod 8 = g, so one twiddled DFT matrix serves them);
    // butterfly j reads x[j + 128 r].
    v4f yre[2], yim[2];
#pragma unroll
    for (int gg = 0; gg < 2; gg++) {
        const uint32_t* rb = X + c.oRB + gg;
        uint32_t w[8];
#pragma unroll
        for (int i = 0; i < 8; i++)
            w[i] = rb[144 * i];
        const Op8 bo = gather_op(w, c.sel);
        const v4f z = {0.f, 0.f, 0.f, 0.f};
        yre[gg] = mfma(c.a_re[gg], bo, z);
        yim[gg] = mfma(c.a_im[gg], bo, z);
    }
    // outputs Y[m] of butterfly j = g + 8 n to d = 128 n + g + 8 m, times pass C's twiddle
#pragma unroll
    for (int gg = 0; gg < 2; gg++) {
        uint32_t* wb = Y + c.oWB + gg;
        cf t = c.twBase[gg];  // w_2048^{n (g + 8 m)}, m = 4 kq + i: twBase w_256^{n i}
        // opaque per transform, so the products below are not hoisted out of
        // the transform loop (that would hold all eight in registers again)
        asm volatile("" : "+v"(t.x), "+v"(t.y));
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const cf y = cmul(cf{yre[gg][i], yim[gg][i]}, t);
            wb[8 * i] = pack_f16(y.x, y.y);
            if (i < 3)
                t = cmul(t, c.twStep);
        }
    }
    // the next transform's maximum, from its raw words (loaded a transform
    // and a half ago, so the wait for them is short)
    publish_max<BF>(c, nxt, red);
    __syncthreads();

    // the next transform's exponent and pass-A operand words
    e_max = block_exponent(red);
    scale_operands<BF>(nxt, op, 4 - e_max);
    pin(op);

    // ---- pass C: radix 16 (NS = 128) on MFMA over butterflies j = 16 g + n,
    // natural-order outputs d = j + 128 m.  The product is taken transposed,
    // Y^T = X^T F^T (the data as the A operand, the DFT matrix as B: the same
    // registers as Y = F X with the operands swapped), so a lane's four
    // accumulators are outputs m = lane % 16 of the consecutive butterflies
    // n = 4 (lane / 16) + i: four consecutive elements.
#pragma unroll
    for (int gg = 0; gg < 2; gg++) {
        const uint32_t* rc = Y + c.oRC + 16 * gg;
        uint32_t w[8];
#pragma unroll
        for (int i = 0; i < 8; i++)
            w[i] = rc[130 * i];
        const Op8 bo = gather_op(w, c.sel);
        const v4f z = {0.f, 0.f, 0.f, 0.f};
        yre[gg] = mfma(bo, c.f_re, z);
        yim[gg] = mfma(bo, c.f_im, z);
    }
    // Lane (m, q) of wave w holds elements 128 m + 32 w + 16 gg + 4 q + i:
    // the wave owns rows m = 0..15 of a 32-element (128-byte) column strip.
    // Stored as they are, consecutive lanes would write different lines.
    // The strip goes through a wavefront-private LDS area instead (rows of
    // 36 words, conflict-free for the writes), and is read back so that
    // lanes 8 r' .. 8 r' + 7 hold row r' in order: each group of 8 lanes then
    // stores one whole line.  The area lies in this wave's own part of the
    // A -> B buffer (plus padding no wave uses): no other wave touches it
    // before the next transform's first barrier, which this wave reaches
    // only after its reads.
    uint32_t* sw = X + STAGE_WAVE * c.wave;
#pragma unroll
    for (int gg = 0; gg < 2; gg++) {
        v4u o;
        if (out_exp) {  // block floating point: the exponent carries the scale
#pragma unroll
            for (int i = 0; i < 4; i++)
                o[i] = pack_store<BF>(yre[gg][i], yim[gg][i]);
        } else {  // unit scale: the exponent applied to each value
#pragma unroll
            for (int i = 0; i < 4; i++)
                o[i] = pack_store<BF>(ldexpf(yre[gg][i], e_out), ldexpf(yim[gg][i], e_out));
        }
        *reinterpret_cast<v4u*>(sw + c.oStW + 16 * gg) = o;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    gu4* dst = reinterpret_cast<gu4*>(out + b * HN + c.oSt);
#pragma unroll
    for (int h = 0; h < 2; h++)
        __builtin_nontemporal_store(*reinterpret_cast<const v4u*>(sw + c.oStR + STAGE_ROW * 8 * h), dst + 256 * h);
    if (out_exp && c.tid == 0)
        out_exp[b] = e_out;
}

// Persistent: a workgroup walks transforms blockIdx.x, + gridDim.x, ...,
// with the inputs of the next two transforms loaded ahead while one is
// computed: two raw register buffers, the loop unrolled twice so each
// body's buffer roles are fixed.  One set of LDS exchange buffers and
// per-wave maxima serves every transform.
template <int S, bool BF>
__global__ __launch_bounds__(HWG, 4) void k_fft_half_2048(const uint32_t* __restrict__ in,
                                                       const int32_t* __restrict__ in_exp,
                                                       uint32_t* __restrict__ out, int32_t* __restrict__ out_exp,
                                                       const cf* __restrict__ tw, int64_t batch, int scale_log2)
{
    __shared__ __align__(16) uint32_t ldsX[BUFA];
    __shared__ __align__(16) uint32_t ldsY[BUFB];
    __shared__ float s_red[HWG / 64];
    int64_t b = blockIdx.x;
    if (b >= batch)
        return;
    HalfCtx c;
    c.tid = threadIdx.x;
    c.lane = c.tid & 63;
    c.wave = c.tid >> 6;
    const int n = c.lane & 15, kq = c.lane >> 4, r0 = (kq & 1) * 8;
    c.f8 = dft8_operand<S>(c.lane, tw);
    dft16_operands<S>(c.f_re, c.f_im, c.lane, 0, tw);
#pragma unroll
    for (int gg = 0; gg < 2; gg++) {
        const int g = 2 * c.wave + gg;
        dft16_operands<S>(c.a_re[gg], c.a_im[gg], c.lane, g, tw);
        c.twBase[gg] = tw_at<S>(tw, n * (g + 32 * kq));  // w_2048^{n (g + 8 m)} at m = 4 kq
    }
    c.twStep = tw_at<S>(tw, 8 * n);  // w_2048^{8 n}: one step of m
    c.oLd = 64 * c.wave + n + 512 * kq;
    c.oWA = fA(8 * (64 * c.wave + n) + 2 * kq);
    c.oRB = fA(2 * c.wave + 8 * n + 128 * r0);
    c.oWB = fB(128 * n + 2 * c.wave + 32 * kq);
    c.oRC = fB(32 * c.wave + n + 128 * r0);
    c.sel = (kq >> 1) ? 0x07060302u : 0x05040100u;  // rows k >= 16 take the imaginary halves
    c.oStW = STAGE_ROW * n + 4 * kq;                                // row m = lane % 16, quad lane / 16
    c.oStR = STAGE_ROW * (c.lane >> 3) + 4 * (c.lane & 7);         // row lane / 8, quad lane % 8
    c.oSt = 128 * (c.lane >> 3) + 32 * c.wave + 4 * (c.lane & 7);  // its element of the output

    // two raw buffers: loading three or four transforms ahead measured no
    // faster (MI355X, 32768 transforms: 93-95 us for each depth)
    constexpr int D = 2;
    uint32_t u[D][8], op[8];
    const int64_t stride = gridDim.x;
#pragma unroll
    for (int r = 0; r < D; r++)
        load_raw(u[r], in, b + r * stride < batch ? b + r * stride : batch - 1, c.oLd);
    publish_max<BF>(c, u[0], s_red);
    __syncthreads();
    int e_max = block_exponent(s_red);
    scale_operands<BF>(u[0], op, 4 - e_max);
    pin(op);
    while (true) {
#pragma unroll
        for (int r = 0; r < D; r++) {
            half_transform<S, BF>(c, op, e_max, u[r], u[(r + 1) % D], ldsX, ldsY, s_red, in, in_exp, out, out_exp,
                                  b, b + D * stride, batch, scale_log2);
            b += stride;
            if (b >= batch)
                return;
        }
    }
}

template <int S, bool BF>
hipError_t launch_half(const void* in, const int32_t* in_exp, void* out, int32_t* out_exp, const void* tw,
                       int64_t batch, int scale_log2, int64_t grid_limit, hipStream_t stream)
{
    const int64_t grid = grid_limit > 0 && batch > grid_limit ? grid_limit : batch;
    return launch_kernel((k_fft_half_2048<S, BF>), dim3((unsigned)grid), dim3(HWG), 0, stream,
                       static_cast<const uint32_t*>(in), in_exp, static_cast<uint32_t*>(out), out_exp,
                       static_cast<const cf*>(tw), batch, scale_log2);
}

template <int S, bool BF>
int occupancy_half()
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_fft_half_2048<S, BF>, HWG, 0) != hipSuccess)
        return 0;
    return blocks;
}

thread_local char g_hmsg[256] = "";

std::vector<KernelHalfSmall>& small_reg()
{
    static std::vector<KernelHalfSmall> r;
    return r;
}

const KernelHalfSmall* find_small(int log2n, int sign, bool bf16)
{
    for (const auto& k : small_reg())
        if (k.log2n == log2n && k.sign == sign && k.bf16 == bf16)
            return &k;
    return nullptr;
}

int ilog2h(int64_t v)
{
    int l = 0;
    while ((int64_t(1) << l) < v)
        l++;
    return l;
}

}  // namespace

hipError_t launch_twiddle_rows(const void* tw, void* rows, int L, int E, int total, hipStream_t stream);

void register_half_small(const KernelHalfSmall& k) { small_reg().push_back(k); }

struct HalfPlan {
    int64_t n = 0, batch = 0;
    int dtype = FFT_C16;
    int64_t grid_limit[2] = {0, 0};  // CUs x resident workgroups, forward / inverse kernel
    const KernelHalfSmall* small[2] = {nullptr, nullptr};  // n < 2048: forward / inverse kernel
    void* rows = nullptr;                                  // their twiddle rows
};

bool half_supported(int64_t n) { return n >= 2 && n <= HN && (n & (n - 1)) == 0; }
const char* half_supported_lengths() { return "2, 4, ..., 2048"; }
const char* half_last_message() { return g_hmsg; }

int half_create(HalfPlan** out, int64_t n, int64_t batch, int dtype, const void* tw)
{
    *out = nullptr;
    if (batch > 0x7fffffffLL) {
        snprintf(g_hmsg, sizeof g_hmsg, "batch=%lld exceeds one launch", (long long)batch);
        return FFT_EINVAL_BATCH;
    }
    auto* hp = new (std::nothrow) HalfPlan();
    if (!hp) {
        snprintf(g_hmsg, sizeof g_hmsg, "out of host memory");
        return FFT_ENOMEM;
    }
    hp->n = n;
    hp->batch = batch;
    hp->dtype = dtype;
    if (n < HN) {
        const int L = ilog2h(n);
        const bool bf = dtype == FFT_CBF16;
        hp->small[0] = find_small(L, -1, bf);
        hp->small[1] = find_small(L, +1, bf);
        if (!hp->small[0] || !hp->small[1]) {
            snprintf(g_hmsg, sizeof g_hmsg, "no half-precision kernel for n=%lld", (long long)n);
            delete hp;
            return FFT_EINVAL_CONFIG;
        }
        const KernelHalfSmall* k = hp->small[0];
        if (k->rows > 0) {
            hipError_t e = hipMalloc(&hp->rows, (size_t)k->rows * sizeof(float2));
            if (e == hipSuccess)
                e = launch_twiddle_rows(tw, hp->rows, L, k->log2ept, k->rows, nullptr);
            if (e == hipSuccess)
                e = hipStreamSynchronize(nullptr);
            if (e != hipSuccess) {
                snprintf(g_hmsg, sizeof g_hmsg, "half-precision twiddle rows: %s", hipGetErrorString(e));
                half_destroy(hp);
                return e == hipErrorOutOfMemory ? FFT_ENOMEM : FFT_EHIP;
            }
        }
        *out = hp;
        return FFT_OK;
    }
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        snprintf(g_hmsg, sizeof g_hmsg, "cannot query the device's compute units");
        delete hp;
        return FFT_EHIP;
    }
    const int occ_f = dtype == FFT_CBF16 ? occupancy_half<-1, true>() : occupancy_half<-1, false>();
    const int occ_i = dtype == FFT_CBF16 ? occupancy_half<1, true>() : occupancy_half<1, false>();
    hp->grid_limit[0] = (int64_t)cus * std::max(occ_f, 1);
    hp->grid_limit[1] = (int64_t)cus * std::max(occ_i, 1);
    *out = hp;
    return FFT_OK;
}

int half_execute(HalfPlan* hp, const void* in, const int32_t* in_exp, void* out, int32_t* out_exp, const void* tw,
                 int sign, bool inv_scale, hipStream_t stream)
{
    hipError_t e;
    // the 1/N of an inverse-scaled transform, exact in the exponent
    const int sl = inv_scale ? -ilog2h(hp->n) : 0;
    if (hp->small[0]) {
        e = hp->small[sign > 0 ? 1 : 0]->fn(in, in_exp, out, out_exp, hp->rows, hp->batch, sl, stream);
        if (e != hipSuccess) {
            snprintf(g_hmsg, sizeof g_hmsg, "half-precision kernel launch: %s", hipGetErrorString(e));
            return FFT_EHIP;
        }
        return FFT_OK;
    }
    const bool bf = hp->dtype == FFT_CBF16;
    if (sign < 0)
        e = bf ? launch_half<-1, true>(in, in_exp, out, out_exp, tw, hp->batch, sl, hp->grid_limit[0], stream)
               : launch_half<-1, false>(in, in_exp, out, out_exp, tw, hp->batch, sl, hp->grid_limit[0], stream);
    else
        e = bf ? launch_half<+1, true>(in, in_exp, out, out_exp, tw, hp->batch, sl, hp->grid_limit[1], stream)
               : launch_half<+1, false>(in, in_exp, out, out_exp, tw, hp->batch, sl, hp->grid_limit[1], stream);
    if (e != hipSuccess) {
        snprintf(g_hmsg, sizeof g_hmsg, "half-precision kernel launch: %s", hipGetErrorString(e));
        return FFT_EHIP;
    }
    return FFT_OK;
}

void half_destroy(HalfPlan* hp)
{
    if (hp && hp->rows)
        (void)hipFree(hp->rows);
    delete hp;
}

void half_query(int64_t n, int64_t batch, fft_plan_desc* d)
{
    if (n < HN) {
        const KernelHalfSmall* k = find_small(ilog2h(n), -1, false);
        d->n = n;
        d->batch = batch;
        if (!k)
            return;
        const int L = ilog2h(n), tpt = (int)(n >> k->log2ept);
        d->ept = 1 << k->log2ept;
        d->wg = k->wg;
        d->transforms_per_wg = k->wg / tpt;
        d->grid = (batch + d->transforms_per_wg - 1) / d->transforms_per_wg;
        if (k->grid_cap > 0 && d->grid > k->grid_cap)
            d->grid = k->grid_cap;  // the launch's cap: workgroups loop over groups
        const int rem = L % k->log2ept;
        int np = 0;
        if (rem)
            d->radices[np++] = 1 << rem;
        for (int i = 0; i < L / k->log2ept; i++)
            d->radices[np++] = 1 << k->log2ept;
        d->npasses = np;
        d->kind = 0;
        d->variant = 0;
        return;
    }
    d->n = n;
    d->batch = batch;
    d->ept = 8;
    d->wg = HWG;
    d->transforms_per_wg = 1;
    d->grid = batch;
    d->npasses = 3;
    d->radices[0] = 8;
    d->radices[1] = 16;
    d->radices[2] = 16;
    d->lds_bytes = (int)((BUFA + BUFB) * sizeof(uint32_t) + 2 * HWG / 64 * sizeof(float));
    d->kind = 0;
    d->variant = 0;
}

void half_describe(const HalfPlan* hp, fft_plan_desc* d)
{
    half_query(hp->n, hp->batch, d);
    if (hp->small[0])
        return;
    const int64_t lim = hp->grid_limit[d->sign > 0 ? 1 : 0];
    if (lim > 0 && d->grid > lim)
        d->grid = lim;
}

}  // namespace mifft
