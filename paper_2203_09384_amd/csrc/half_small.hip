// FP16 / BF16 storage for lengths 2 .. 1024 (compiled once per log2 N with
// -DMIFFT_LOG2N=<1..10>): block floating point around the FP32 Stockham
// passes of the batched kernels.
//
// Storage is (re, im) pairs of 16-bit values with one int32 exponent per
// transform (logical value = stored * 2^exp).  Each transform is
//   loaded and widened to FP32, scaled by the power of two that brings its
//   largest component into [1/2, 1) (exact), transformed with the FP32
//   passes (growth at most N <= 2^10), scaled again so its largest output
//   component lies in [2^14, 2^15) (exact), and narrowed to the storage
//   type once.
// out_exp = in_exp + e_in + e_out - 15 (- log2 N for the inverse's 1/N).
// The radix-16 MFMA passes of the 2048-point kernel need at least 256
// points and pay off at that size; here the transform's threads share one
// wavefront, so both maxima are wavefront shuffles.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_fft.hpp"
#include "launch.hpp"
#include "half.hpp"

#ifndef MIFFT_LOG2N
#error "compile with -DMIFFT_LOG2N=<1..10>"
#endif

namespace mifft {
namespace {

typedef unsigned int v4u __attribute__((ext_vector_type(4)));

template <bool BF>
__device__ __forceinline__ float h_to_f32(uint32_t h)
{
    if constexpr (BF)
        return __builtin_bit_cast(float, h << 16);
    else
        return (float)__builtin_bit_cast(_Float16, (uint16_t)h);
}

template <bool BF>
__device__ __forceinline__ uint32_t f32_to_h(float f)
{
    if constexpr (BF)
        return (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)f);
    else
        return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)f);
}

// Largest |component| over the TPT threads of a transform (contiguous
// lanes of one wavefront), in every one of them.
template <int TPT>
__device__ __forceinline__ float group_max(float m)
{
#pragma unroll
    for (int off = TPT / 2; off > 0; off >>= 1)
        m = fmaxf(m, __shfl_xor(m, off));
    return m;
}

template <int E>
__device__ __forceinline__ float abs_max(const cf (&v)[1 << E])
{
    float m = 0.f;
#pragma unroll
    for (int i = 0; i < (1 << E); i++)
        m = fmaxf(m, fmaxf(fabsf(v[i].x), fabsf(v[i].y)));
    return m;
}

// the exponent e with m < 2^e (0 for zero or non-finite m)
__device__ __forceinline__ int exp_above(float m)
{
    int e = 0;
    if (m > 0.f && m <= 3.4e38f)
        (void)frexpf(m, &e);
    return e;
}

// Lengths 2^3..2^10 launch a capped grid whose workgroups loop over groups
// of transforms, so each pass's twiddle row is read into registers once per
// workgroup rather than once per group (at 2^26 elements N = 8: 107 -> 93
// us, 16: 107 -> 92, 32: 126 -> 113, 64: 105 -> 94, 128: 114 -> 108, 256:
// 113 -> 104, 512: 114 -> 107, 1024: 145 -> 123 us).  The caps are the
// measured best per length.
template <int L>
constexpr bool small_persistent()
{
    return L >= 3;
}
constexpr int64_t small_persist_grid(int L) { return L == 8 ? 8192 : (L <= 4 || L == 10 ? 16384 : 32768); }

template <int L, int E>
constexpr bool small_staged()
{
    constexpr int EPT = 1 << E;
    return EPT >= 4 && (L <= 6 || L == 10);
}
template <int L, int E>
constexpr int small_roww()
{
    constexpr int N = 1 << L, TPT = N >> E;
    return N + (TPT == 1 ? 0 : (TPT > 4 ? TPT : 4));
}

// One group of TPB transforms (group index g) through the kernel's steps.
template <int L, int E, int WG, int S, bool BF, int TW>
__device__ __forceinline__ void small_group(const uint32_t* __restrict__ in, const int32_t* __restrict__ in_exp,
                                            uint32_t* __restrict__ out, int32_t* __restrict__ out_exp,
                                            const cf* __restrict__ rows, int64_t batch, int scale_log2, int64_t g,
                                            const TwRegs<L, E>& tws, cf* lds, uint32_t* blk)
{
    using SC = Sched<L, E>;
    constexpr int N = SC::N, EPT = SC::EPT, TPT = SC::TPT, TPB = WG / TPT;
    constexpr int REG = TPT > 1 ? Layout2<L, E>::region() : 1;
    const int tid = threadIdx.x, tb = tid / TPT, t = tid % TPT;
    const int64_t first = g * TPB;
    const int64_t b = first + tb;
    const bool live = b < batch;
    // Staged lengths (EPT >= 4; measured faster at N = 4..64 and 1024, slower
    // at 128..512): the workgroup's block of TPB transforms moves between
    // HBM and LDS in 16-byte vectors at consecutive lanes (1 KiB per wave
    // instruction); in LDS each transform is a row of N words padded so
    // that the threads of neighbouring transforms read distinct banks.
    constexpr bool STAGED = small_staged<L, E>();
    constexpr int ROWW = small_roww<L, E>();
    constexpr int K = STAGED ? EPT / 4 : 1;  // 16-byte vectors per thread
    const int64_t count = batch - first < TPB ? batch - first : TPB;
    const int nv = (int)count * (N / 4);
    v4u q[K];
    cf v[EPT];
    if constexpr (STAGED) {
        const gu4* src = reinterpret_cast<const gu4*>(in + first * N);
        if (count == TPB) {
#pragma unroll
            for (int k = 0; k < K; k++)
                q[k] = __builtin_nontemporal_load(src + tid + WG * k);
        } else {
#pragma unroll
            for (int k = 0; k < K; k++)
                q[k] = tid + WG * k < nv ? __builtin_nontemporal_load(src + tid + WG * k) : v4u{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int k = 0; k < K; k++) {
            const int w = 4 * (tid + WG * k);  // first word of the vector in the block
            *reinterpret_cast<v4u*>(blk + (w / N) * ROWW + w % N) = q[k];
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < EPT; m++) {
            const uint32_t u = blk[tb * ROWW + t + m * TPT];
            v[m] = cf{h_to_f32<BF>(u & 0xffffu), h_to_f32<BF>(u >> 16)};
        }
    } else {
#pragma unroll
        for (int m = 0; m < EPT; m++) {
            const uint32_t u = live ? in[b * N + t + m * TPT] : 0u;
            v[m] = cf{h_to_f32<BF>(u & 0xffffu), h_to_f32<BF>(u >> 16)};
        }
    }
    // normalise: largest component into [1/2, 1), as an exponent shift of
    // each value (exact, and no overflow of a 2^-e_in factor when the
    // largest component is near the bottom of the format's range)
    const int e_in = exp_above(group_max<TPT>(abs_max<E>(v)));
#pragma unroll
    for (int m = 0; m < EPT; m++)
        v[m] = cf{ldexpf(v[m].x, -e_in), ldexpf(v[m].y, -e_in)};
    if constexpr (TPT == 1)
        pass_compute2<L, E, S, 0>(v, tws[0]);
    else
        run2<L, E, S, TW, true>(v, t, rows, tws, lds + tb * REG);
    // output: largest component into [2^14, 2^15), or the logical value
    const int e_o = exp_above(group_max<TPT>(abs_max<E>(v)));
    const int ein = (live && in_exp) ? in_exp[b] : 0;
    const int e_total = ein + e_in + e_o - 15 + scale_log2;  // logical = stored * 2^e_total
#pragma unroll
    for (int m = 0; m < EPT; m++) {
        const cf y = out_exp ? cf{ldexpf(v[m].x, 15 - e_o), ldexpf(v[m].y, 15 - e_o)}
                             : cf{ldexpf(v[m].x, ein + e_in + scale_log2), ldexpf(v[m].y, ein + e_in + scale_log2)};
        const uint32_t u = f32_to_h<BF>(y.x) | (f32_to_h<BF>(y.y) << 16);
        if constexpr (STAGED)
            blk[tb * ROWW + t + m * TPT] = u;  // this thread's own elements: no other thread reads them yet
        else if (live)
            out[b * N + t + m * TPT] = u;
    }
    if (out_exp && live && t == 0)
        out_exp[b] = e_total;
    if constexpr (STAGED) {
        __syncthreads();
        gu4* dst = reinterpret_cast<gu4*>(out + first * N);
#pragma unroll
        for (int k = 0; k < K; k++) {
            const int w = 4 * (tid + WG * k);
            q[k] = *reinterpret_cast<const v4u*>(blk + (w / N) * ROWW + w % N);
        }
        if (count == TPB) {
#pragma unroll
            for (int k = 0; k < K; k++)
                __builtin_nontemporal_store(q[k], dst + tid + WG * k);
        } else {
#pragma unroll
            for (int k = 0; k < K; k++)
                if (tid + WG * k < nv)
                    __builtin_nontemporal_store(q[k], dst + tid + WG * k);
        }
    }
}

template <int L, int E, int WG, int S, bool BF>
__global__ __launch_bounds__(WG) void k_half_small(const uint32_t* __restrict__ in, const int32_t* __restrict__ in_exp,
                                                   uint32_t* __restrict__ out, int32_t* __restrict__ out_exp,
                                                   const cf* __restrict__ rows, int64_t batch, int scale_log2)
{
    using SC = Sched<L, E>;
    constexpr int EPT = SC::EPT, TPT = SC::TPT, TPB = WG / TPT;
    static_assert(TPT <= 64, "a transform's threads share one wavefront");
    constexpr int REG = TPT > 1 ? Layout2<L, E>::region() : 1;
    __shared__ cf lds[TPT > 1 ? TPB * REG : 1];
    __shared__ __attribute__((aligned(16))) uint32_t blk[small_staged<L, E>() ? TPB * small_roww<L, E>() : 4];
    TwRegs<L, E> tws;
#pragma unroll
    for (int p = 0; p < SC::NP; p++)
#pragma unroll
        for (int r = 0; r < EPT; r++)
            tws[p][r] = cf{1.f, 0.f};
    if constexpr (small_persistent<L>() && TPT > 1) {
        load_all_rows<L, E, S>(tws, rows, threadIdx.x % TPT);
        const int64_t ngroups = (batch + TPB - 1) / TPB;
        for (int64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
            if (g != blockIdx.x)
                __syncthreads();  // the previous group's block and exchanges are read out
            small_group<L, E, WG, S, BF, 0>(in, in_exp, out, out_exp, rows, batch, scale_log2, g, tws, lds, blk);
        }
    } else {
        small_group<L, E, WG, S, BF, 1>(in, in_exp, out, out_exp, rows, batch, scale_log2, blockIdx.x, tws, lds, blk);
    }
}

template <int L, int E, int WG, int S, bool BF>
hipError_t launch_half_small(const void* in, const int32_t* in_exp, void* out, int32_t* out_exp, const void* rows,
                             int64_t batch, int scale_log2, hipStream_t stream)
{
    constexpr int TPB = WG / ((1 << L) >> E);
    const int64_t ngroups = (batch + TPB - 1) / TPB;
    constexpr int64_t cap = small_persist_grid(L);
    const int64_t grid = small_persistent<L>() && ngroups > cap ? cap : ngroups;
    return launch_kernel((k_half_small<L, E, WG, S, BF>), dim3((unsigned)grid), dim3(WG), 0, stream,
                       static_cast<const uint32_t*>(in), in_exp, static_cast<uint32_t*>(out), out_exp,
                       static_cast<const cf*>(rows), batch, scale_log2);
}

// One configuration per length: elements per thread and workgroup size.
constexpr int small_e(int L) { return L <= 2 ? L : (L <= 5 ? 2 : (L == 6 || L == 7 || L == 9 ? 3 : 4)); }
constexpr int small_wg(int L) { return L <= 2 ? 64 : (L <= 5 || L == 8 ? 256 : 64); }

template <int L>
void add_small()
{
    constexpr int E = small_e(L), WG = small_wg(L), TPT = (1 << L) >> E;
    const int rows = TPT > 1 ? Layout2<L, E>::rows_total() : 0;
    const int64_t cap = small_persistent<L>() ? small_persist_grid(L) : 0;
    register_half_small(KernelHalfSmall{L, E, WG, -1, false, &launch_half_small<L, E, WG, -1, false>, rows, cap});
    register_half_small(KernelHalfSmall{L, E, WG, +1, false, &launch_half_small<L, E, WG, +1, false>, rows, cap});
    register_half_small(KernelHalfSmall{L, E, WG, -1, true, &launch_half_small<L, E, WG, -1, true>, rows, cap});
    register_half_small(KernelHalfSmall{L, E, WG, +1, true, &launch_half_small<L, E, WG, +1, true>, rows, cap});
}

struct HalfSmallRegistrar {
    HalfSmallRegistrar() { add_small<MIFFT_LOG2N>(); }
};
HalfSmallRegistrar half_small_registrar;

}  // namespace
}  // namespace mifft
