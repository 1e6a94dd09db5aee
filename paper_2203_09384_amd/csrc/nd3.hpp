// Host-side registry of the single-pass 3D kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mifft {

// in -> out: `batch` row-major N0 x N1 x N2 arrays, all three axes
// transformed, every output multiplied by scale.  rows: the per-pass
// twiddle rows of the axis-0, axis-1 and axis-2 transforms (2^log2ept
// points per thread) back to back, rows0 + rows1 + rows2 entries.
using LaunchNd3 = hipError_t (*)(const void* in, void* out, const void* rows, int64_t batch, float scale,
                                 hipStream_t stream);

struct KernelNd3 {
    int log2n[3], log2ept, sign;
    int arrays_per_wg, wg;
    LaunchNd3 fn;
    int rows[3];  // twiddle-row entries (float2) of each axis (0 for a one-thread axis)
    int lds_bytes;
    // persistent form: the workgroups resident on the current device at once
    // (its grid; 0 if the query fails), nullptr for one workgroup per group
    int (*slots)();
};

void register_nd3(const KernelNd3& k);
const KernelNd3* find_nd3(int log2n0, int log2n1, int log2n2, int sign);

}  // namespace mifft
