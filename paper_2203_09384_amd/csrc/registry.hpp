// Host-side registry of compiled kernel variants.  Each kernel translation
// unit registers its instantiations at library load; the planner looks
// them up by (log2 N, log2 EPT, workgroup size, sign).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mifft {

// Launch one FP32 batched transform: `batch` transforms of N = 2^log2n
// interleaved complex64 elements from `in` to `out`, output multiplied by
// `scale`.  `tw` is the 2048-entry table exp(-2 pi i m / 2048); `rows` the
// per-pass twiddle rows of the variant (kind >= 1); `grid_limit` > 0 caps
// the workgroup count of persistent kinds.
using LaunchC32 = hipError_t (*)(const void* in, void* out, const void* tw, const void* rows, int64_t batch,
                                 float scale, int64_t grid_limit, hipStream_t stream);

struct KernelC32 {
    int log2n, log2ept, wg, sign;
    int kind;                 // 0: one transform group per workgroup, per-pass table reads
                              // 1..4: twiddle-row kernels (1 + TW + 2 PF), see fft_c32.hip
                              // 5..8: the same with wave-local LDS exchanges
    LaunchC32 fn;
    int (*occupancy)();       // workgroups per CU (persistent kinds), else NULL
    int rows;                 // twiddle-row entries the variant needs (kind >= 1)
    int lds_bytes;            // LDS per workgroup
};

void register_c32(const KernelC32& k);
const KernelC32* find_c32(int log2n, int log2ept, int wg, int sign, int kind);
int count_c32();
const KernelC32* c32_at(int i);

}  // namespace mifft
