// FP16/BF16 path (placeholder until the MFMA kernel lands).
#include "half.hpp"

namespace mifft {
struct HalfPlan {
    int dummy;
};
bool half_supported(int64_t) { return false; }
const char* half_supported_lengths() { return ""; }
int half_create(HalfPlan**, int64_t, int64_t, int) { return FFT_EINVAL_DTYPE; }
int half_execute(HalfPlan*, const void*, const int32_t*, void*, int32_t*, const void*, int, hipStream_t) { return FFT_EINVAL_DTYPE; }
void half_destroy(HalfPlan* hp) { delete hp; }
void half_describe(const HalfPlan*, fft_plan_desc*) {}
void half_query(int64_t, int64_t, fft_plan_desc*) {}
const char* half_last_message() { return "FP16/BF16 plans are not available in this build"; }
}  // namespace mifft
