// A plain streaming copy, the practical HBM ceiling the benchmark reports
// beside the transforms: each thread moves K 16-byte vectors with
// nontemporal loads and stores, consecutive lanes at consecutive addresses
// (1 KiB per wave instruction), the loads of a thread issued before its
// stores.  Several workgroup shapes are compiled; the benchmark reports
// the best.  Measurement support only (not part of the FFT library).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.hpp"

namespace {

typedef uint32_t u4 __attribute__((ext_vector_type(4)));

template <int WG, int K>
__global__ __launch_bounds__(WG) void k_stream_copy(const u4* __restrict__ in, u4* __restrict__ out, int64_t nvec)
{
    const int64_t base = (int64_t)blockIdx.x * (WG * K) + threadIdx.x;
    u4 q[K];
    if (base + (int64_t)(K - 1) * WG < nvec) {
#pragma unroll
        for (int k = 0; k < K; k++)
            q[k] = __builtin_nontemporal_load(in + base + k * WG);
#pragma unroll
        for (int k = 0; k < K; k++)
            __builtin_nontemporal_store(q[k], out + base + k * WG);
    } else {
#pragma unroll
        for (int k = 0; k < K; k++)
            if (base + k * WG < nvec)
                __builtin_nontemporal_store(__builtin_nontemporal_load(in + base + k * WG), out + base + k * WG);
    }
}

template <int WG, int K>
hipError_t run(const void* in, void* out, int64_t nvec, hipStream_t st)
{
    const int64_t grid = (nvec + WG * K - 1) / (WG * K);
    return mifft::launch_kernel(k_stream_copy<WG, K>, dim3((unsigned)grid), dim3(WG), 0, st,
                                static_cast<const u4*>(in), static_cast<u4*>(out), nvec);
}

}  // namespace

extern "C" {

// Number of compiled shapes and the (workgroup size, vectors per thread) of shape i.
int stream_copy_shapes(void) { return 5; }
int stream_copy_shape(int i, int* wg, int* k)
{
    static const int s[5][2] = {{64, 1}, {256, 1}, {256, 2}, {256, 4}, {512, 2}};
    if (i < 0 || i >= 5)
        return -1;
    *wg = s[i][0];
    *k = s[i][1];
    return 0;
}

// Copy `bytes` (a multiple of 16; both pointers 16-byte aligned) with shape i.
int stream_copy(const void* in, void* out, int64_t bytes, int i, void* stream)
{
    if (bytes <= 0 || (bytes & 15) || ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15))
        return -1;
    const int64_t nvec = bytes / 16;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e;
    switch (i) {
    case 0: e = run<64, 1>(in, out, nvec, st); break;
    case 1: e = run<256, 1>(in, out, nvec, st); break;
    case 2: e = run<256, 2>(in, out, nvec, st); break;
    case 3: e = run<256, 4>(in, out, nvec, st); break;
    case 4: e = run<512, 2>(in, out, nvec, st); break;
    default: return -1;
    }
    return e == hipSuccess ? 0 : (int)e;
}

}  // extern "C"
