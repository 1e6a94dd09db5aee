// Host-side registry of the axis kernels of multidimensional plans.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mifft {

// In place on `io`: `count` transforms of length 2^log2n along an axis of
// stride 2^log2s elements; transform q starts at element
// (q >> log2s) * 2^(log2n + log2s) + (q & (2^log2s - 1)).  rows: the
// transform's per-pass twiddle rows; every output is multiplied by scale.
using LaunchAxis = hipError_t (*)(void* io, const void* rows, int64_t count, int log2s, float scale,
                                  hipStream_t stream);

struct KernelAxis {
    int log2n;
    int log2ept;
    int sign;
    int tile;  // transforms per workgroup
    LaunchAxis fn;
    int rows;       // twiddle-row entries (float2)
    int lds_bytes;
};

void register_axis(const KernelAxis& k);
const KernelAxis* find_axis(int log2n, int sign);

}  // namespace mifft
