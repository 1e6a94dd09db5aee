// FP16 / BF16 storage path: block floating point; N = 2048 with radix-16
// stages on MFMA, N = 2 .. 1024 around the FP32 Stockham passes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mifft.h"

namespace mifft {

struct HalfPlan;

// Lengths 2 .. 1024 (half_small.hip): rows are the per-pass twiddle rows of
// (log2n, log2ept); scale_log2 is added to every output exponent.
using LaunchHalfSmall = hipError_t (*)(const void* in, const int32_t* in_exp, void* out, int32_t* out_exp,
                                       const void* rows, int64_t batch, int scale_log2, hipStream_t stream);
struct KernelHalfSmall {
    int log2n, log2ept, wg, sign;
    bool bf16;
    LaunchHalfSmall fn;
    int rows;          // twiddle-row entries (float2)
    int64_t grid_cap;  // > 0: at most this many workgroups, each looping over groups of transforms
};
void register_half_small(const KernelHalfSmall& k);

bool half_supported(int64_t n);
const char* half_supported_lengths();
int half_create(HalfPlan** out, int64_t n, int64_t batch, int dtype, const void* tw);
// sign: the exponent sign applied; inv_scale: whether the 1/N is applied
// (the plan's scale, also for its adjoint, which has the opposite sign).
int half_execute(HalfPlan* hp, const void* in, const int32_t* in_exp, void* out, int32_t* out_exp,
                 const void* tw, int sign, bool inv_scale, hipStream_t stream);
void half_destroy(HalfPlan* hp);
void half_describe(const HalfPlan* hp, fft_plan_desc* d);
void half_query(int64_t n, int64_t batch, fft_plan_desc* d);
const char* half_last_message();

}  // namespace mifft
