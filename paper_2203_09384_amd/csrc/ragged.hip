// Ragged batches (placeholder until the persistent kernel lands).
#include "ragged.hpp"
#include "../../include/mifft.h"

namespace mifft {
struct RaggedPlan {
    int dummy;
};
int ragged_check_config(const int*, int, int) { return FFT_OK; }
int ragged_create(RaggedPlan**, int64_t, const int64_t*, const int*, int, int, int) { return FFT_EINVAL_DTYPE; }
int ragged_execute(RaggedPlan*, const void*, void*, const void*, int, bool, hipStream_t) { return FFT_EINVAL_DTYPE; }
void ragged_destroy(RaggedPlan* rp) { delete rp; }
void ragged_describe(const RaggedPlan*, int*, int64_t*, int64_t*, int*) {}
const char* ragged_last_message() { return "ragged plans are not available in this build"; }
}  // namespace mifft
