// FP16 / BF16 storage path, N = 2048: block floating point, radix-16 stages
// as dense 16 x 16 complex DFT-matrix products on MFMA.
//
// The paper's library is FP32-only (section "Implementation"); this path
// stores data as half-precision (re, im) pairs and computes the same DFT of
// Eq. (dft) with the Cooley-Tukey split 2048 = 8 * 16 * 16:
//   pass A  radix-8 butterflies on the VALU in FP32 (no twiddles, NS = 1)
//   pass B  radix-16 (NS = 8)   } Y = F16 X for 16 butterflies at a time,
//   pass C  radix-16 (NS = 128) } F16 the 16-point DFT matrix,
// where each complex product is two real MFMAs over K = 32:
//   Re Y = [Re F | -Im F] [Re X; Im X],   Im Y = [Im F | Re F] [Re X; Im X]
// on v_mfma_f32_16x16x32_f16 with FP32 accumulation.  The
// inter-pass twiddles (FP32, from the plan's table) are applied when a pass
// writes its outputs to LDS, so every MFMA operand is a plain gather.
//
// Block floating point: logical value = stored * 2^exp[b] per transform.
// On load the transform is scaled by a power of two so its largest
// component lies in [8, 16); with the at most 8 * 16 * 16 = 2^11 growth of
// the three passes no operand can exceed 2^15 < 65504, and the output is
// stored at that scale with exponent in_exp + e_max - 4 (- 11 for the
// inverse's 1/N, exact).  Scaling is by powers of two only, so it adds no
// rounding.
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
typedef float v4f __attribute__((ext_vector_type(4)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

constexpr int HN = 2048;
constexpr int HWG = 256;

// LDS layouts, one per exchange, each conflict-free for both its writer and
// its reader (modelled on the 64 banks) and affine in the per-instruction
// indices, so every access is a per-thread base plus an immediate offset.
// Element d is one 32-bit word holding its (re, im) as two 16-bit halves:
// FP16 for the A -> B and B -> C exchanges (the MFMA operand type, so
// rounding there is the operands' own rounding), the storage format for
// C -> store (output scale applied first, so the value is rounded once).
//   A -> B      : d + (d >> 3) + 16 (d >> 10)
//   B -> C      : d + (d >> 6)
//   C -> store  : d + (d >> 6) + 4 (d >> 8)
__device__ __forceinline__ int fA(int d) { return d + (d >> 3) + 16 * (d >> 10); }
__device__ __forceinline__ int fB(int d) { return d + (d >> 6); }
__device__ __forceinline__ int fC(int d) { return d + (d >> 6) + 4 * (d >> 8); }
constexpr int BUF = 2336;  // words per buffer (largest layout: fA)

// ---- conversions (round to nearest even)
template <bool BF>
__device__ __forceinline__ float to_f32(uint16_t h)
{
    if constexpr (BF)
        return __builtin_bit_cast(float, (uint32_t)h << 16);
    else
        return (float)__builtin_bit_cast(_Float16, h);
}
template <bool BF>
__device__ __forceinline__ uint16_t from_f32(float f)
{
    if constexpr (BF)
        return __builtin_bit_cast(uint16_t, (__bf16)f);
    else
        return __builtin_bit_cast(uint16_t, (_Float16)f);
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

template <int S>
__device__ __forceinline__ cf tw_at(const cf* __restrict__ tw, int idx)
{
    cf w = tw[idx];
    if constexpr (S > 0)
        w.y = -w.y;
    return w;
}

template <bool BF>
__device__ __forceinline__ void unpack8(const uint32_t (&u)[8], cf (&v)[8])
{
#pragma unroll
    for (int m = 0; m < 8; m++)
        v[m] = cf{to_f32<BF>((uint16_t)(u[m] & 0xffffu)), to_f32<BF>((uint16_t)(u[m] >> 16))};
}

// Per-thread constants of the kernel: MFMA operands, twiddles, LDS bases.
struct HalfCtx {
    Op8 a_re[2], a_im[2];  // pass B, group g = 2 wave + gg, twiddles folded
    Op8 f_re, f_im;        // pass C, plain DFT
    cf twB[2][4];          // pass C twiddle of pass B output (gg, i)
    int oWA, oRB[2], oWB[2], oRC[2], oWC[2], oRS0, oRS1;
    uint32_t sel;          // byte selector of this lane's halves (re: low, im: high)
    int tid, lane, wave;
};

// Two floats to one word of two halves (a low, b high), each rounded to
// nearest even: one packed convert (v_cvt_pk_f16_f32 / v_cvt_pk_bf16_f32).
typedef float v2f32 __attribute__((ext_vector_type(2)));
typedef _Float16 v2f16 __attribute__((ext_vector_type(2)));
typedef __bf16 v2bf16 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pack_f16(float a, float b)
{
    const v2f32 f = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, v2f16));
}

template <bool BF>
__device__ __forceinline__ uint32_t pack_store(float a, float b)
{
    const v2f32 f = {a, b};
    if constexpr (BF)
        return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, v2bf16));
    else
        return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, v2f16));
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

__device__ __forceinline__ void load_raw(uint32_t (&u)[8], const uint32_t* __restrict__ in, int64_t b, int tid)
{
    const uint32_t* src = in + b * HN;
#pragma unroll
    for (int m = 0; m < 8; m++)
        u[m] = __builtin_nontemporal_load(src + tid + 256 * m);
}

// One transform: raw input `cur` (thread t holds x[t + 256 m]) -> stored
// output and exponent.  Once unpacked, `cur` is refilled with transform
// `refill` (if < batch), so two transforms' loads stay in flight.  X holds
// the A->B and C->store exchanges, Y the B->C exchange; `red` the per-wave
// maxima.  Four barriers: the block maximum (needed before pass A's
// outputs are scaled to FP16), then one per exchange.
template <int S, bool BF>
__device__ __forceinline__ void half_transform(const HalfCtx& c, uint32_t (&cur)[8], uint32_t* X, uint32_t* Y,
                                               float* red, const uint32_t* __restrict__ in,
                                               const int32_t* __restrict__ in_exp, uint32_t* __restrict__ out,
                                               int32_t* __restrict__ out_exp, int64_t b, int64_t refill,
                                               int scale_log2)
{
    constexpr int dWC[4] = {0, 130, 264, 394};  // fC(d0 + 128 i) - fC(d0)
    // ---- pass A: radix 8 on the VALU in FP32 over x[tid + 256 m]
    cf v[8];
    unpack8<BF>(cur, v);
    // This transform's input exponent is read before the refill is issued,
    // and the refill itself is unconditional (past the end of the batch it
    // re-reads the last transform, which every workgroup shares through
    // the cache): a load issued after the refill, or a refill under a
    // condition, would make the first wait below cover the refill as well.
    const int e_in = in_exp ? in_exp[b] : 0;
    load_raw(cur, in, refill, c.tid);
    float mx = 0.f;
#pragma unroll
    for (int m = 0; m < 8; m++)
        mx = fmaxf(mx, fmaxf(fabsf(v[m].x), fabsf(v[m].y)));
    mx = wave_max_nonneg(mx);
    if (c.lane == 0)
        red[c.wave] = mx;
    dft8<S>(v);
    __syncthreads();

    // ---- block maximum -> power-of-two scale (largest input component in [8, 16))
    mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    int e_max = 0;
    if (mx > 0.f && mx <= 3.4e38f)
        (void)frexpf(mx, &e_max);  // mx < 2^e_max
    // applied as an exponent shift of each value (v_ldexp_f32): exact, and
    // unlike a multiply by 2^(4 - e_max) it cannot overflow when the
    // transform's largest component is near the bottom of the format's range
    const int sh = 4 - e_max;
    const int e_out = e_in + e_max - 4 + scale_log2;
    // outputs to the Stockham position d = 8 tid + r, scaled, as FP16 pairs
    // (pass B's twiddles are in its operands)
    uint32_t* wa = X + c.oWA;
#pragma unroll
    for (int r = 0; r < 8; r++)
        wa[r] = pack_f16(ldexpf(v[r].x, sh), ldexpf(v[r].y, sh));
    __syncthreads();

    // ---- pass B: radix 16 (NS = 8) on MFMA.  Group g holds the 16 butterflies
    // j = g + 8 n (all with j mod 8 = g, so one twiddled DFT matrix serves them);
    // butterfly j reads x[j + 128 r].
    v4f yre[2], yim[2];
#pragma unroll
    for (int gg = 0; gg < 2; gg++) {
        const uint32_t* rb = X + c.oRB[gg];
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
        uint32_t* wb = Y + c.oWB[gg];
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const cf y = cmul(cf{yre[gg][i], yim[gg][i]}, c.twB[gg][i]);
            wb[8 * i] = pack_f16(y.x, y.y);
        }
    }
    __syncthreads();

    // ---- pass C: radix 16 (NS = 128) on MFMA over butterflies j = 16 g + n;
    // natural-order outputs d = j + 128 m, stored in the output format
#pragma unroll
    for (int gg = 0; gg < 2; gg++) {
        const uint32_t* rc = Y + c.oRC[gg];
        uint32_t w[8];
#pragma unroll
        for (int i = 0; i < 8; i++)
            w[i] = rc[130 * i];
        const Op8 bo = gather_op(w, c.sel);
        const v4f z = {0.f, 0.f, 0.f, 0.f};
        yre[gg] = mfma(c.f_re, bo, z);
        yim[gg] = mfma(c.f_im, bo, z);
    }
    if (out_exp) {  // block floating point: the exponent carries the scale
#pragma unroll
        for (int gg = 0; gg < 2; gg++) {
            uint32_t* wc = X + c.oWC[gg];
#pragma unroll
            for (int i = 0; i < 4; i++)
                wc[dWC[i]] = pack_store<BF>(yre[gg][i], yim[gg][i]);
        }
    } else {  // unit scale: the exponent applied to each value
#pragma unroll
        for (int gg = 0; gg < 2; gg++) {
            uint32_t* wc = X + c.oWC[gg];
#pragma unroll
            for (int i = 0; i < 4; i++)
                wc[dWC[i]] = pack_store<BF>(ldexpf(yre[gg][i], e_out), ldexpf(yim[gg][i], e_out));
        }
    }
    __syncthreads();

    // ---- store: 4 consecutive elements (16 bytes) per lane and instruction
    gu4* dst = reinterpret_cast<gu4*>(out + b * HN);
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const uint32_t* rs = X + (h ? c.oRS1 : c.oRS0);
        v4u o;
#pragma unroll
        for (int i = 0; i < 4; i++)
            o[i] = rs[i];
        __builtin_nontemporal_store(o, dst + c.tid + HWG * h);
    }
    if (out_exp && c.tid == 0)
        out_exp[b] = e_out;
}

// This thread's LDS bases and byte selector.
__device__ __forceinline__ void init_offsets(HalfCtx& c)
{
    c.tid = threadIdx.x;
    c.lane = c.tid & 63;
    c.wave = c.tid >> 6;
    const int n = c.lane & 15, kq = c.lane >> 4, r0 = (kq & 1) * 8;
#pragma unroll
    for (int gg = 0; gg < 2; gg++) {
        const int g = 2 * c.wave + gg;
        c.oRB[gg] = fA(g + 8 * n + 128 * r0);
        c.oWB[gg] = fB(128 * n + g + 32 * kq);
        const int j = 16 * g + n;
        c.oRC[gg] = fB(j + 128 * r0);
        c.oWC[gg] = fC(j + 512 * kq);
    }
    c.sel = (kq >> 1) ? 0x07060302u : 0x05040100u;  // rows k >= 16 take the imaginary halves
    c.oWA = fA(8 * c.tid);
    c.oRS0 = fC(4 * c.tid);
    c.oRS1 = fC(4 * (c.tid + HWG));
}

// The per-thread constants: MFMA operands and twiddles gathered from the
// FP32 twiddle table, LDS bases.
template <int S>
__device__ __forceinline__ void init_ctx(HalfCtx& c, const cf* __restrict__ tw)
{
    init_offsets(c);
    const int n = c.lane & 15, kq = c.lane >> 4;
    dft16_operands<S>(c.f_re, c.f_im, c.lane, 0, tw);
#pragma unroll
    for (int gg = 0; gg < 2; gg++) {
        const int g = 2 * c.wave + gg;
        dft16_operands<S>(c.a_re[gg], c.a_im[gg], c.lane, g, tw);
#pragma unroll
        for (int i = 0; i < 4; i++)  // w_2048^{n (g + 8 m)}, m = 4 kq + i
            c.twB[gg][i] = tw_at<S>(tw, n * (g + 8 * (4 * kq + i)));
    }
}

// The same constants as a table of CTX_VEC 16-byte words per thread, word k
// of thread t at tab[k HWG + t] (coalesced loads): the operands f_re, f_im,
// a_re[0], a_im[0], a_re[1], a_im[1], then twB[gg][2h], twB[gg][2h + 1] for
// (gg, h) = (0, 0), (0, 1), (1, 0), (1, 1).  Built once per plan by
// k_half_ctx_table from the gathers above, so both routes hold the same bits.
constexpr int CTX_VEC = 10;

__device__ __forceinline__ v4u cf2_word(cf a, cf b)
{
    return v4u{__builtin_bit_cast(uint32_t, a.x), __builtin_bit_cast(uint32_t, a.y), __builtin_bit_cast(uint32_t, b.x),
               __builtin_bit_cast(uint32_t, b.y)};
}

template <int S>
__global__ __launch_bounds__(HWG) void k_half_ctx_table(const cf* __restrict__ tw, v4u* __restrict__ tab)
{
    HalfCtx c;
    init_ctx<S>(c, tw);
    v4u* t = tab + c.tid;
    t[0 * HWG] = __builtin_bit_cast(v4u, c.f_re.hi);
    t[1 * HWG] = __builtin_bit_cast(v4u, c.f_im.hi);
#pragma unroll
    for (int gg = 0; gg < 2; gg++) {
        t[(2 + 2 * gg) * HWG] = __builtin_bit_cast(v4u, c.a_re[gg].hi);
        t[(3 + 2 * gg) * HWG] = __builtin_bit_cast(v4u, c.a_im[gg].hi);
#pragma unroll
        for (int h = 0; h < 2; h++)
            t[(6 + 2 * gg + h) * HWG] = cf2_word(c.twB[gg][2 * h], c.twB[gg][2 * h + 1]);
    }
}

// (Elements are copied out before the bit casts: a bit cast applied to a
// vector element expression directly has been seen to read element 0.)
__device__ __forceinline__ cf word_cf(const v4u& w, int h)
{
    const uint32_t re = w[2 * h], im = w[2 * h + 1];
    return cf{__builtin_bit_cast(float, re), __builtin_bit_cast(float, im)};
}

__device__ __forceinline__ void load_ctx(HalfCtx& c, const v4u* __restrict__ tab)
{
    init_offsets(c);
    v4u q[CTX_VEC];
#pragma unroll
    for (int k = 0; k < CTX_VEC; k++)
        q[k] = tab[k * HWG + c.tid];
    c.f_re.hi = __builtin_bit_cast(v8h, q[0]);
    c.f_im.hi = __builtin_bit_cast(v8h, q[1]);
#pragma unroll
    for (int gg = 0; gg < 2; gg++) {
        c.a_re[gg].hi = __builtin_bit_cast(v8h, q[2 + 2 * gg]);
        c.a_im[gg].hi = __builtin_bit_cast(v8h, q[3 + 2 * gg]);
#pragma unroll
        for (int h = 0; h < 2; h++) {
            c.twB[gg][2 * h] = word_cf(q[6 + 2 * gg + h], 0);
            c.twB[gg][2 * h + 1] = word_cf(q[6 + 2 * gg + h], 1);
        }
    }
}

// Transforms per workgroup.  Measured at N = 2048, batch 32768 with the
// input streamed from HBM: 4 (and 8) beat both shorter runs (1, 2: too
// little in flight per workgroup) and a persistent grid of CUs x 4
// workgroups looping over the batch (about 10% slower: the same copy
// pattern without any arithmetic loses as much against a one-shot grid).
constexpr int64_t kRun = 4;

// A workgroup takes `per_wg` consecutive transforms (the last workgroup
// fewer), with the inputs of the next two in flight while one is computed.
// Past the end of its run the refill re-reads the batch's last transform,
// which every workgroup shares through the cache, so the refill stays
// unconditional.  Two LDS buffers (and two raw register buffers) alternate
// between consecutive transforms (loop unrolled twice so each body's
// buffer roles are fixed), so three barriers suffice.
template <int S, bool BF>
__global__ __launch_bounds__(HWG, 4) void k_fft_half_2048(const uint32_t* __restrict__ in,
                                                       const int32_t* __restrict__ in_exp,
                                                       uint32_t* __restrict__ out, int32_t* __restrict__ out_exp,
                                                       const v4u* __restrict__ ctab, int64_t batch, int64_t per_wg,
                                                       int scale_log2)
{
    __shared__ uint32_t lds[2 * BUF];
    __shared__ float s_red[2][HWG / 64];
    int64_t b = (int64_t)blockIdx.x * per_wg;
    const int64_t end = b + per_wg < batch ? b + per_wg : batch;
    const int64_t last = batch - 1;
    uint32_t ua[8], ub[8];
    load_raw(ua, in, b, threadIdx.x);
    load_raw(ub, in, b + 1 < end ? b + 1 : last, threadIdx.x);
    __builtin_amdgcn_sched_barrier(0);  // the first transform's loads are issued before the second's
    HalfCtx c;
    load_ctx(c, ctab);
    uint32_t* const buf0 = lds;
    uint32_t* const buf1 = lds + BUF;
    while (true) {
        half_transform<S, BF>(c, ua, buf0, buf1, s_red[0], in, in_exp, out, out_exp, b, b + 2 < end ? b + 2 : last,
                              scale_log2);
        if (++b >= end)
            break;
        half_transform<S, BF>(c, ub, buf1, buf0, s_red[1], in, in_exp, out, out_exp, b, b + 2 < end ? b + 2 : last,
                              scale_log2);
        if (++b >= end)
            break;
    }
}

// Largest grid of one launch: 2^32 - 1 work-items of HWG threads.
constexpr int64_t kMaxGrid = (((int64_t)1 << 32) - 1) / HWG;

// Transforms per workgroup: kRun, more only when the batch would need a
// grid beyond one launch's limit.
int64_t half_run_length(int64_t batch)
{
    return (batch + kRun - 1) / kRun > kMaxGrid ? (batch + kMaxGrid - 1) / kMaxGrid : kRun;
}

template <int S, bool BF>
hipError_t launch_half(const void* in, const int32_t* in_exp, void* out, int32_t* out_exp, const void* ctab,
                       int64_t batch, int scale_log2, hipStream_t stream)
{
    const int64_t per_wg = half_run_length(batch);
    const int64_t grid = (batch + per_wg - 1) / per_wg;
    return launch_kernel((k_fft_half_2048<S, BF>), dim3((unsigned)grid), dim3(HWG), 0, stream,
                         static_cast<const uint32_t*>(in), in_exp, static_cast<uint32_t*>(out), out_exp,
                         static_cast<const v4u*>(ctab), batch, per_wg, scale_log2);
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
    const KernelHalfSmall* small[2] = {nullptr, nullptr};  // n < 2048: forward / inverse kernel
    void* rows = nullptr;                                  // their twiddle rows
    void* ctx = nullptr;  // n = 2048: per-thread constant tables, forward then inverse
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
    const size_t tab = (size_t)CTX_VEC * HWG * sizeof(v4u);
    hipError_t e = hipMalloc(&hp->ctx, 2 * tab);
    if (e == hipSuccess)
        e = launch_kernel(k_half_ctx_table<-1>, dim3(1), dim3(HWG), 0, nullptr, static_cast<const cf*>(tw),
                          static_cast<v4u*>(hp->ctx));
    if (e == hipSuccess)
        e = launch_kernel(k_half_ctx_table<1>, dim3(1), dim3(HWG), 0, nullptr, static_cast<const cf*>(tw),
                          static_cast<v4u*>(hp->ctx) + CTX_VEC * HWG);
    if (e == hipSuccess)
        e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        snprintf(g_hmsg, sizeof g_hmsg, "half-precision constant tables: %s", hipGetErrorString(e));
        half_destroy(hp);
        return e == hipErrorOutOfMemory ? FFT_ENOMEM : FFT_EHIP;
    }
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
    const v4u* ctab = static_cast<const v4u*>(hp->ctx) + (sign > 0 ? CTX_VEC * HWG : 0);
    if (sign < 0)
        e = bf ? launch_half<-1, true>(in, in_exp, out, out_exp, ctab, hp->batch, sl, stream)
               : launch_half<-1, false>(in, in_exp, out, out_exp, ctab, hp->batch, sl, stream);
    else
        e = bf ? launch_half<+1, true>(in, in_exp, out, out_exp, ctab, hp->batch, sl, stream)
               : launch_half<+1, false>(in, in_exp, out, out_exp, ctab, hp->batch, sl, stream);
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
    if (hp && hp->ctx)
        (void)hipFree(hp->ctx);
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
    d->transforms_per_wg = (int)half_run_length(batch);
    d->grid = (batch + d->transforms_per_wg - 1) / d->transforms_per_wg;
    d->npasses = 3;
    d->radices[0] = 8;
    d->radices[1] = 16;
    d->radices[2] = 16;
    d->lds_bytes = (int)(2 * BUF * sizeof(uint32_t) + 2 * HWG / 64 * sizeof(float));
    d->kind = 0;
    d->variant = 0;
}

void half_describe(const HalfPlan* hp, fft_plan_desc* d) { half_query(hp->n, hp->batch, d); }

}  // namespace mifft
