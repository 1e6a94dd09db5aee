// Registry of the four-step kernels for FP32 lengths 2^12 .. 2^20.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mifft {

// Launch both passes: in -> out (pass 1), out in place (pass 2).
using LaunchFourStep = hipError_t (*)(const void* in, void* out, const void* rows1, const void* rows2,
                                      const void* tlo, const void* thi, int64_t batch, float scale,
                                      hipStream_t stream);

struct FourStep {
    int log2n, log2n1, log2n2;  // N = N1 * N2, column length N1, row length N2
    int log2e1, log2e2;         // elements per thread of the inner transforms
    int rows1, rows2;           // twiddle-row entries of the inner transforms
    LaunchFourStep fwd, bwd;    // sign -1 / +1
    int lds1, lds2;             // LDS per workgroup of each pass
    int tile1;                  // columns per pass-1 workgroup
};

void register_fourstep(const FourStep& f);
const FourStep* find_fourstep(int log2n);
hipError_t launch_twiddle_big(void* lo, void* hi, int L, hipStream_t stream);

}  // namespace mifft
