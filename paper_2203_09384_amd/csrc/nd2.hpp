// Host-side registry of the single-pass 2D kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mifft {

// in -> out: `batch` row-major N0 x N1 arrays, both axes transformed, every
// output multiplied by scale.  rows0 / rows1: per-pass twiddle rows of the
// column (2^log2n0) and row (2^log2n1) transforms at 2^log2ept points per
// thread.
using LaunchNd2 = hipError_t (*)(const void* in, void* out, const void* rows0, const void* rows1, int64_t batch,
                                 float scale, hipStream_t stream);

struct KernelNd2 {
    int log2n0, log2n1, log2ept, sign;
    int arrays_per_wg, wg;
    LaunchNd2 fn;
    int rows0, rows1;  // twiddle-row entries (float2)
    int lds_bytes;
    // persistent form: the workgroups resident on the current device at once
    // (its grid; 0 if the query fails), nullptr for one workgroup per group
    int (*slots)();
};

void register_nd2(const KernelNd2& k);
const KernelNd2* find_nd2(int log2n0, int log2n1, int sign);

}  // namespace mifft
