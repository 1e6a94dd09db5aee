// Ragged (mixed-length) batches: plan-side tile list and the persistent kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mifft {

struct RaggedPlan;

// Checks a forced per-length variant table (NULL = built-in choice).
int ragged_check_config(const int* ept_by_log2n, int wg, int ctas_per_cu);
// Builds the tile list from host `offsets` (already validated) and uploads it.
// `tw` is the plan's 2048-entry twiddle table (device).
int ragged_create(RaggedPlan** out, int64_t count, const int64_t* offsets, const int* ept_by_log2n, int wg,
                  int ctas_per_cu, int device, const void* tw);
// One persistent launch over every tile.  sign: exponent sign applied;
// inverse_scale: multiply each transform by 1/its length.
int ragged_execute(RaggedPlan* rp, const void* in, void* out, const void* tw, int sign, bool inverse_scale,
                   hipStream_t stream);
void ragged_destroy(RaggedPlan* rp);
void ragged_describe(const RaggedPlan* rp, int* wg, int64_t* grid, int64_t* tiles, int* lds_bytes,
                     int* ept_by_log2n);
const char* ragged_last_message();

}  // namespace mifft
