// Registry of the fused loss-and-gradient kernels (fused_loss.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mifft {

// loss[b] = sum_k w |(A x_b)_k|^2 and grad_b = A^H (2 w A x_b) for the
// batched FP32 transform A of sign `sign` and scale `scale`.
using LaunchLossGrad = hipError_t (*)(const void* x, const float* w, void* grad, float* loss, const void* rows,
                                      int64_t batch, float scale, int64_t grid_limit, hipStream_t stream);

struct KernelLossGrad {
    int log2n, log2ept, wg, sign;
    LaunchLossGrad fn;
    int (*occupancy)();
    int rows;  // twiddle-row entries needed (0: one thread per transform)
};

void register_loss_grad(const KernelLossGrad& k);
const KernelLossGrad* find_loss_grad(int log2n, int log2ept, int wg, int sign);

}  // namespace mifft
