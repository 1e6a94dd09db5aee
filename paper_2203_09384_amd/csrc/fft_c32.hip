// FP32 interleaved complex batched Stockham FFT kernels, one translation
// unit per transform length: this file is compiled once per log2(N) with
// -DMIFFT_LOG2N=<1..11> and registers every (EPT, workgroup size, sign)
// variant it instantiates with the host-side kernel registry.
//
// Workgroup layout: TPT = N/EPT threads per transform, TPB = WG/TPT
// transforms per workgroup, one transform per TPT consecutive threads.
// Thread t of a transform loads x[t + m TPT] for m < EPT (each wave load
// instruction covers whole 64-lane runs of consecutive complex values),
// runs every pass in registers with LDS exchanges in between, and stores
// X[t + m TPT] (natural order), multiplied by the plan's scale.
#include "device_fft.hpp"
#include "registry.hpp"

#ifndef MIFFT_LOG2N
#error "compile with -DMIFFT_LOG2N=<1..11>"
#endif

namespace mifft {
namespace {

template <int LOG2N, int LOG2EPT, int WG, int S>
__global__ __launch_bounds__(WG) void k_fft_c32(const cf* __restrict__ in, cf* __restrict__ out,
                                                const cf* __restrict__ tw, int64_t batch, float scale)
{
    using SC = Sched<LOG2N, LOG2EPT>;
    constexpr int N = SC::N, EPT = SC::EPT, TPT = SC::TPT, TPB = WG / TPT;
    const int tid = threadIdx.x;
    const int tb = tid / TPT, t = tid % TPT;
    const int64_t b = (int64_t)blockIdx.x * TPB + tb;
    const bool live = b < batch;
    const cf* __restrict__ src = in + b * N;
    cf* __restrict__ dst = out + b * N;
    cf v[EPT];

    if constexpr (TPT == 1) {
        // One thread owns a whole (short) transform: 16-byte vector loads of
        // consecutive elements, a single in-register DFT, no LDS.
        static_assert(SC::NP == 1, "single pass expected");
        if (live) {
            const float4* s4 = reinterpret_cast<const float4*>(src);
#pragma unroll
            for (int m = 0; m < EPT / 2; m++) {
                const float4 q = s4[m];
                v[2 * m] = cf{q.x, q.y};
                v[2 * m + 1] = cf{q.z, q.w};
            }
        } else {
#pragma unroll
            for (int m = 0; m < EPT; m++)
                v[m] = cf{0.f, 0.f};
        }
        pass_compute<LOG2N, LOG2EPT, S, 0>(v, 0, tw);
        if (live) {
            float4* d4 = reinterpret_cast<float4*>(dst);
#pragma unroll
            for (int m = 0; m < EPT / 2; m++)
                d4[m] = float4{v[2 * m].x * scale, v[2 * m].y * scale, v[2 * m + 1].x * scale,
                               v[2 * m + 1].y * scale};
        }
    } else {
        __shared__ float lre[TPB * N];
        __shared__ float lim[TPB * N];
#pragma unroll
        for (int m = 0; m < EPT; m++)
            v[m] = live ? src[t + m * TPT] : cf{0.f, 0.f};
        run_passes<LOG2N, LOG2EPT, S>(v, t, tw, lre + tb * N, lim + tb * N);
        if (live) {
#pragma unroll
            for (int m = 0; m < EPT; m++)
                dst[t + m * TPT] = cscale(v[m], scale);
        }
    }
}

template <int LOG2N, int LOG2EPT, int WG, int S>
hipError_t launch_c32(const void* in, void* out, const void* tw, int64_t batch, float scale,
                      hipStream_t stream)
{
    constexpr int TPB = WG / Sched<LOG2N, LOG2EPT>::TPT;
    const int64_t grid = (batch + TPB - 1) / TPB;
    hipLaunchKernelGGL((k_fft_c32<LOG2N, LOG2EPT, WG, S>), dim3((unsigned)grid), dim3(WG), 0, stream,
                       static_cast<const cf*>(in), static_cast<cf*>(out), static_cast<const cf*>(tw),
                       batch, scale);
    return hipGetLastError();
}

// Variant menu: EPT in {2,4,8,16} (not above N; at least 4 once N >= 64),
// WG in {64,128,256,512}, TPT <= WG, LDS per workgroup <= 64 KiB; a thread
// owns a whole transform (TPT = 1) only for N <= 16.
template <int LOG2N, int LOG2EPT, int WG>
constexpr bool valid_cfg()
{
    if (LOG2EPT > LOG2N) return false;
    if (LOG2N >= 6 && LOG2EPT < 2) return false;
    constexpr int TPT = (1 << LOG2N) >> LOG2EPT;
    if (TPT > WG) return false;
    if (TPT == 1 && LOG2N > 4) return false;
    if (TPT > 1 && (WG << LOG2EPT) * 8 > 65536) return false;
    return true;
}

template <int LOG2N, int LOG2EPT, int WG, int S>
void add_one()
{
    if constexpr (valid_cfg<LOG2N, LOG2EPT, WG>())
        register_c32(KernelC32{LOG2N, LOG2EPT, WG, S, &launch_c32<LOG2N, LOG2EPT, WG, S>});
}

template <int LOG2N, int LOG2EPT>
void add_wgs()
{
    add_one<LOG2N, LOG2EPT, 64, -1>();
    add_one<LOG2N, LOG2EPT, 64, +1>();
    add_one<LOG2N, LOG2EPT, 128, -1>();
    add_one<LOG2N, LOG2EPT, 128, +1>();
    add_one<LOG2N, LOG2EPT, 256, -1>();
    add_one<LOG2N, LOG2EPT, 256, +1>();
    add_one<LOG2N, LOG2EPT, 512, -1>();
    add_one<LOG2N, LOG2EPT, 512, +1>();
}

struct Registrar {
    Registrar()
    {
        add_wgs<MIFFT_LOG2N, 1>();
        add_wgs<MIFFT_LOG2N, 2>();
        add_wgs<MIFFT_LOG2N, 3>();
        add_wgs<MIFFT_LOG2N, 4>();
    }
};
Registrar registrar;

}  // namespace
}  // namespace mifft
