// Host-side registry of the real-input (FFT_R32) kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mifft {

// in/out: device buffers (real n values or n/2+1 complex bins per transform,
// by direction); rows: per-pass twiddle rows of the half-length transform;
// wn: w_n^k for k < n/2.  we / wi: weights of the edge bins (0, n/2) and of
// the interior bins (see real.hip).  grid_limit: workgroups of a persistent
// launch (0 = one per transform group).
using LaunchReal = hipError_t (*)(const void* in, void* out, const void* rows, const void* wn, int64_t batch,
                                  float we, float wi, int64_t grid_limit, hipStream_t stream);

struct KernelReal {
    int log2m;    // log2 of the half length n/2 (0..14)
    int log2ept;  // complex elements per thread of the half-length transform
    int wg;
    int dir;      // 0: real -> bins (R2C), 1: bins -> real (C2R)
    int kind;     // 0: a whole half-length transform per thread; else as FP32 variants 1..8
    LaunchReal fn;
    int (*occupancy)();
    int rows;       // twiddle-row entries (float2) the kernel reads
    int lds_bytes;  // LDS per workgroup
};

void register_real(const KernelReal& k);
const KernelReal* find_real(int log2m, int log2ept, int wg, int dir, int kind);

hipError_t launch_twiddle_real(const void* tw, void* wn, int log2n, hipStream_t stream);

}  // namespace mifft

namespace mifft {

// Real-input lengths above 2^15: the even/odd split as a pass of its own
// around a four-step complex transform of the half length M = n/2.
//   dir 0: src = Z (M complex per transform), dst = bins X_0..X_M
//   dir 1: src = bins X_0..X_M, dst = Z' (M complex per transform)
// tlo / thi: the two-level table w_n^j = thi[j >> 10] * tlo[j & 1023].
hipError_t launch_real_split(int dir, const void* src, void* dst, const void* tlo, const void* thi, int log2n,
                             int64_t batch, float we, float wi, hipStream_t stream);

}  // namespace mifft
