// Host-side registry of compiled kernel variants.  Each kernel translation
// unit registers its instantiations at library load; the planner looks
// them up by (log2 N, log2 EPT, workgroup size, sign).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mifft {

// Launch one FP32 batched transform: `batch` transforms of N = 2^log2n
// interleaved complex64 elements from `in` to `out`, twiddle table `tw`
// (2048 entries exp(-2 pi i m / 2048)), output multiplied by `scale`.
using LaunchC32 = hipError_t (*)(const void* in, void* out, const void* tw, int64_t batch, float scale,
                                 hipStream_t stream);

struct KernelC32 {
    int log2n, log2ept, wg, sign;
    LaunchC32 fn;
};

void register_c32(const KernelC32& k);
const KernelC32* find_c32(int log2n, int log2ept, int wg, int sign);
int count_c32();
const KernelC32* c32_at(int i);

}  // namespace mifft
