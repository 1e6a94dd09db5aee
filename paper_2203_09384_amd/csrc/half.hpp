// FP16 / BF16 storage path: block floating point, radix-16 stages on MFMA.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mifft.h"

namespace mifft {

struct HalfPlan;

bool half_supported(int64_t n);
const char* half_supported_lengths();
int half_create(HalfPlan** out, int64_t n, int64_t batch, int dtype);
int half_execute(HalfPlan* hp, const void* in, const int32_t* in_exp, void* out, int32_t* out_exp,
                 const void* tw, int sign, hipStream_t stream);
void half_destroy(HalfPlan* hp);
void half_describe(const HalfPlan* hp, fft_plan_desc* d);
void half_query(int64_t n, int64_t batch, fft_plan_desc* d);
const char* half_last_message();

}  // namespace mifft
