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
// on v_mfma_f32_16x16x32_{f16,bf16} with FP32 accumulation.  The
// inter-pass twiddles (FP32, from the plan's table) are applied when a pass
// writes its outputs to LDS, so every MFMA operand is a plain gather.
//
// Block floating point: logical value = stored * 2^exp[b] per transform.
// On load the transform is scaled by a power of two so its largest
// component lies in [8, 16); with the at most 8 * 16 * 16 = 2^11 growth of
// the three passes no FP16 operand can exceed 2^15 < 65504, and the output
// is stored at that scale with exponent in_exp + e_max - 4 (- 11 for the
// inverse's 1/N, exact).  Scaling is by powers of two only, so it adds no
// rounding.  BF16 operands are split hi + lo (x = hi + lo, both BF16) and
// each real product is Fhi Xhi + Fhi Xlo + Flo Xhi, giving ~16 significant
// bits per operand; FP16 operands are used as is.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_fft.hpp"
#include "half.hpp"

namespace mifft {
namespace {

typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

constexpr int HN = 2048;
constexpr int HWG = 256;
// LDS planes: index i -> i + 16 (i >> 10); the imaginary plane starts 32
// banks after the real one, so the four 16-lane groups of an MFMA operand
// gather hit disjoint banks.
constexpr int PLANE = HN + 16 + 16;
constexpr int IM_OFF = PLANE + 32 - (PLANE % 64);

__device__ __forceinline__ int hp(int i) { return i + ((i >> 10) << 4); }

// ---- conversions (round to nearest even) ----
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f)
{
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_bits_to_f32(uint16_t h)
{
    return __builtin_bit_cast(float, (uint32_t)h << 16);
}
__device__ __forceinline__ uint16_t f32_to_f16_bits(float f)
{
    return __builtin_bit_cast(uint16_t, (_Float16)f);
}
__device__ __forceinline__ float f16_bits_to_f32(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }

template <bool BF>
__device__ __forceinline__ float to_f32(uint16_t h)
{
    if constexpr (BF)
        return bf16_bits_to_f32(h);
    else
        return f16_bits_to_f32(h);
}
template <bool BF>
__device__ __forceinline__ uint16_t from_f32(float f)
{
    if constexpr (BF)
        return f32_to_bf16_bits(f);
    else
        return f32_to_f16_bits(f);
}

// MFMA operand of 8 values (hi part, and for BF16 the lo remainder).
template <bool BF>
struct Op8;
template <>
struct Op8<false> {
    v8h hi;
    __device__ __forceinline__ void set(int i, float x) { hi[i] = (_Float16)x; }
};
template <>
struct Op8<true> {
    v8bf hi, lo;
    __device__ __forceinline__ void set(int i, float x)
    {
        const uint16_t h = f32_to_bf16_bits(x);
        hi[i] = __builtin_bit_cast(__bf16, h);
        lo[i] = __builtin_bit_cast(__bf16, f32_to_bf16_bits(x - bf16_bits_to_f32(h)));
    }
};

__device__ __forceinline__ v4f mfma(const Op8<false>& a, const Op8<false>& b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a.hi, b.hi, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma(const Op8<true>& a, const Op8<true>& b, v4f c)
{
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.hi, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.lo, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.lo, b.hi, c, 0, 0, 0);
}

// This lane's rows of the two A operands: A_re[m] = [Re F[m][.] | -Im F[m][.]],
// A_im[m] = [Im F[m][.] | Re F[m][.]], F[m][r] = exp(S 2 pi i m r / 16);
// lane l holds row m = l % 16, columns k = 8 (l / 16) + i.
template <int S, bool BF>
__device__ __forceinline__ void dft16_operands(Op8<BF>& are, Op8<BF>& aim, int lane)
{
    const int m = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        const int r = (kq & 1) * 8 + i;
        const int e = (m * r) & 15;
        const float c = kCos16[e], s = (float)S * kSin16[e];
        if (kq < 2) {
            are.set(i, c);
            aim.set(i, s);
        } else {
            are.set(i, -s);
            aim.set(i, c);
        }
    }
}

// One radix-16 pass on MFMA over the 128 butterflies of the transform in
// LDS (butterfly j reads x[j + 128 r], r < 16).  Wave w handles butterfly
// groups 2w and 2w+1 (16 butterflies each).  Returns, per group, the lane's
// 4 outputs Y[m], m = 4 (lane / 16) + i, of butterfly j = 16 g + lane % 16.
template <bool BF>
__device__ __forceinline__ void mfma_pass(const float* lds, const Op8<BF>& are, const Op8<BF>& aim, int wave,
                                          int lane, v4f (&yre)[2], v4f (&yim)[2])
{
    const int n = lane & 15, kq = lane >> 4;
    const float* plane = lds + ((kq >> 1) ? IM_OFF : 0);
    const int r0 = (kq & 1) * 8;
#pragma unroll
    for (int gg = 0; gg < 2; gg++) {
        const int j = 16 * (2 * wave + gg) + n;
        Op8<BF> b;
#pragma unroll
        for (int i = 0; i < 8; i++)
            b.set(i, plane[hp(j + 128 * (r0 + i))]);
        const v4f z = {0.f, 0.f, 0.f, 0.f};
        yre[gg] = mfma(are, b, z);
        yim[gg] = mfma(aim, b, z);
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

template <int S, bool BF>
__global__ __launch_bounds__(HWG) void k_fft_half_2048(const uint32_t* __restrict__ in,
                                                       const int32_t* __restrict__ in_exp,
                                                       uint32_t* __restrict__ out, int32_t* __restrict__ out_exp,
                                                       const cf* __restrict__ tw, int scale_log2)
{
    __shared__ float lds[IM_OFF + PLANE];
    __shared__ float s_red[HWG / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t b = blockIdx.x;

    // ---- load: thread t holds x[t + 256 m], m < 8 (4-byte pairs, coalesced)
    const uint32_t* src = in + b * HN;
    cf v[8];
    float mx = 0.f;
#pragma unroll
    for (int m = 0; m < 8; m++) {
        const uint32_t u = src[tid + 256 * m];
        v[m] = cf{to_f32<BF>((uint16_t)(u & 0xffffu)), to_f32<BF>((uint16_t)(u >> 16))};
        mx = fmaxf(mx, fmaxf(fabsf(v[m].x), fabsf(v[m].y)));
    }
    // ---- block maximum -> power-of-two scale (largest component in [8, 16))
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        mx = fmaxf(mx, __shfl_xor(mx, off));
    if (lane == 0)
        s_red[wave] = mx;
    __syncthreads();
    mx = fmaxf(fmaxf(s_red[0], s_red[1]), fmaxf(s_red[2], s_red[3]));
    int e_max = 0;
    if (mx > 0.f && mx <= 3.4e38f)
        (void)frexpf(mx, &e_max);  // mx < 2^e_max
    const float sc = ldexpf(1.0f, 4 - e_max);
    const int e_in = in_exp ? in_exp[b] : 0;
    const int e_out = e_in + e_max - 4 + scale_log2;

    // ---- pass A: radix 8 on VALU, FP32; outputs to LDS with pass B's twiddles
#pragma unroll
    for (int m = 0; m < 8; m++)
        v[m] = cscale(v[m], sc);
    dft8<S>(v);
#pragma unroll
    for (int r = 0; r < 8; r++) {
        const int d = tid * 8 + r;               // Stockham destination, NS = 1, R = 8
        const int jb = d & 127, rb = d >> 7;     // pass B: d = j + 128 r, k = j mod 8
        const cf w = tw_at<S>(tw, (rb * (jb & 7)) << 4);
        const cf y = cmul(v[r], w);
        lds[hp(d)] = y.x;
        lds[IM_OFF + hp(d)] = y.y;
    }
    __syncthreads();

    Op8<BF> are, aim;
    dft16_operands<S, BF>(are, aim, lane);
    const int n = lane & 15, kq = lane >> 4;
    v4f yre[2], yim[2];

    // ---- pass B: radix 16 on MFMA (NS = 8); outputs with pass C's twiddles
    mfma_pass<BF>(lds, are, aim, wave, lane, yre, yim);
    __syncthreads();
#pragma unroll
    for (int gg = 0; gg < 2; gg++) {
        const int j = 16 * (2 * wave + gg) + n;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int m = 4 * kq + i;
            const int d = ((j >> 3) << 7) + (j & 7) + 8 * m;  // Stockham destination, NS = 8
            const int jc = d & 127, rc = d >> 7;              // pass C: d = j + 128 r, k = j
            const cf w = tw_at<S>(tw, rc * jc);
            const cf y = cmul(cf{yre[gg][i], yim[gg][i]}, w);
            lds[hp(d)] = y.x;
            lds[IM_OFF + hp(d)] = y.y;
        }
    }
    __syncthreads();

    // ---- pass C: radix 16 on MFMA (NS = 128); natural-order outputs
    mfma_pass<BF>(lds, are, aim, wave, lane, yre, yim);
    __syncthreads();
#pragma unroll
    for (int gg = 0; gg < 2; gg++) {
        const int j = 16 * (2 * wave + gg) + n;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int d = j + 128 * (4 * kq + i);
            lds[hp(d)] = yre[gg][i];
            lds[IM_OFF + hp(d)] = yim[gg][i];
        }
    }
    __syncthreads();

    // ---- store: 4 consecutive elements (16 bytes) per lane and instruction
    const float osc = out_exp ? 1.0f : ldexpf(1.0f, e_out);
    v4u* dst = reinterpret_cast<v4u*>(out + b * HN);
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const int q = tid + HWG * h;  // 16-byte chunk index, 512 per transform
        v4u o;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int d = 4 * q + i;
            const float re = lds[hp(d)] * osc, im = lds[IM_OFF + hp(d)] * osc;
            o[i] = (uint32_t)from_f32<BF>(re) | ((uint32_t)from_f32<BF>(im) << 16);
        }
        dst[q] = o;
    }
    if (out_exp && tid == 0)
        out_exp[b] = e_out;
}

template <int S, bool BF>
hipError_t launch_half(const void* in, const int32_t* in_exp, void* out, int32_t* out_exp, const void* tw,
                       int64_t batch, int scale_log2, hipStream_t stream)
{
    hipLaunchKernelGGL((k_fft_half_2048<S, BF>), dim3((unsigned)batch), dim3(HWG), 0, stream,
                       static_cast<const uint32_t*>(in), in_exp, static_cast<uint32_t*>(out), out_exp,
                       static_cast<const cf*>(tw), scale_log2);
    return hipGetLastError();
}

thread_local char g_hmsg[256] = "";

}  // namespace

struct HalfPlan {
    int64_t n = 0, batch = 0;
    int dtype = FFT_C16;
};

bool half_supported(int64_t n) { return n == HN; }
const char* half_supported_lengths() { return "2048"; }
const char* half_last_message() { return g_hmsg; }

int half_create(HalfPlan** out, int64_t n, int64_t batch, int dtype)
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
    *out = hp;
    return FFT_OK;
}

int half_execute(HalfPlan* hp, const void* in, const int32_t* in_exp, void* out, int32_t* out_exp, const void* tw,
                 int sign, hipStream_t stream)
{
    const int sl = sign > 0 ? -11 : 0;  // inverse: the 1/N of Eq. (idft), exact in the exponent
    hipError_t e;
    const bool bf = hp->dtype == FFT_CBF16;
    if (sign < 0)
        e = bf ? launch_half<-1, true>(in, in_exp, out, out_exp, tw, hp->batch, sl, stream)
               : launch_half<-1, false>(in, in_exp, out, out_exp, tw, hp->batch, sl, stream);
    else
        e = bf ? launch_half<+1, true>(in, in_exp, out, out_exp, tw, hp->batch, sl, stream)
               : launch_half<+1, false>(in, in_exp, out, out_exp, tw, hp->batch, sl, stream);
    if (e != hipSuccess) {
        snprintf(g_hmsg, sizeof g_hmsg, "half-precision kernel launch: %s", hipGetErrorString(e));
        return FFT_EHIP;
    }
    return FFT_OK;
}

void half_destroy(HalfPlan* hp) { delete hp; }

void half_query(int64_t n, int64_t batch, fft_plan_desc* d)
{
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
    d->lds_bytes = (int)((IM_OFF + PLANE + HWG / 64) * sizeof(float));
    d->kind = 0;
    d->variant = 0;
}

void half_describe(const HalfPlan* hp, fft_plan_desc* d) { half_query(hp->n, hp->batch, d); }

}  // namespace mifft
