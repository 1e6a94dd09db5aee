// Fused weighted spectral power loss and its gradient, one translation unit
// per transform length (-DMIFFT_LOG2N=<1..11>).
//
// For the plan's transform A (sign S, scale c) and weights w >= 0:
//   loss[b] = sum_k w[b,k] |(A x_b)_k|^2
//   grad_b  = A^H (2 w_b * A x_b)         (A^H: sign -S, same scale c)
// which is the gradient of sum_b loss[b] in PyTorch's convention for complex
// inputs (dL/dRe x + i dL/dIm x).  One pass over HBM: x and w are read once,
// grad is written once; the forward result never leaves registers -- after
// the forward passes a thread holds X[t + m N/EPT], exactly the layout the
// adjoint's first pass loads.
#include "device_fft.hpp"
#include "launch.hpp"
#include "fused_loss.hpp"

#ifndef MIFFT_LOG2N
#error "compile with -DMIFFT_LOG2N=<1..11>"
#endif

namespace mifft {
namespace {

template <int L, int E, int TPB>
__device__ __forceinline__ void load_weights(float (&wv)[1 << E], const float* __restrict__ w, int64_t g,
                                             int64_t batch, int tb, unsigned toff4)
{
    using SC = Sched<L, E>;
    constexpr int N = SC::N, EPT = SC::EPT, TPT = SC::TPT;
    constexpr bool NT = TPT >= 32;
    const int64_t first = g * TPB;
    const char* gb = reinterpret_cast<const char*>(w + first * N);
    unsigned off = toff4;
    if constexpr (TPB > 1) {
        // threads of a transform past the end of the batch read the last
        // transform's weights (their loss and gradient are not stored), so
        // that every thread issues the same loads with no branch around them
        const int64_t last = batch - 1 - first;
        off = first + tb < batch ? toff4 : (unsigned)(last * N + (toff4 / 4u) % (unsigned)TPT) * 4u;
    }
#pragma unroll
    for (int m = 0; m < EPT; m++) {
        const float* p = reinterpret_cast<const float*>(gb + (off + (unsigned)(m * TPT * 4)));
        if constexpr (NT)
            wv[m] = __builtin_nontemporal_load(p);
        else
            wv[m] = *p;
    }
}

// Sum of `part` over the TPT <= 64 threads of each transform (one
// wavefront); the total is valid in thread t == 0 of the transform.
template <int TPT>
__device__ __forceinline__ float transform_sum(float part)
{
    static_assert(TPT <= 64, "transforms spanning wavefronts sum through LDS in loss_grad_group");
#pragma unroll
    for (int off = TPT / 2; off > 0; off >>= 1)
        part += __shfl_xor(part, off);
    return part;
}

template <int L, int E, int S>
__device__ __forceinline__ void transform_passes(cf (&v)[1 << E], int t, const cf* __restrict__ rows, cf* lds)
{
    using SC = Sched<L, E>;
    TwRegs<L, E> tws;
#pragma unroll
    for (int p = 0; p < SC::NP; p++)
#pragma unroll
        for (int r = 0; r < SC::EPT; r++)
            tws[p][r] = cf{1.f, 0.f};
    if constexpr (SC::TPT == 1)
        pass_compute2<L, E, S, 0>(v, tws[0]);
    else
        run2<L, E, S, 1, (SC::TPT <= 64)>(v, t, rows, tws, lds);
}

// The forward passes of a group, loading the next group `gn` into `nx` a
// slice per pass (PF), or not at all.
template <int L, int E, int S, int TPB, bool PF>
__device__ __forceinline__ void forward_passes(cf (&v)[1 << E], int t, const cf* __restrict__ rows, cf* lds,
                                               cf (&nx)[1 << E], const cf* __restrict__ x, int64_t gn,
                                               int64_t batch, int tb, unsigned toff8)
{
    using SC = Sched<L, E>;
    if constexpr (!PF) {
        transform_passes<L, E, S>(v, t, rows, lds);
    } else if constexpr (SC::TPT == 1) {
        load_group<L, E, TPB>(nx, x, gn, batch, tb, toff8);
        transform_passes<L, E, S>(v, t, rows, lds);
    } else {
        TwRegs<L, E> tws;
#pragma unroll
        for (int p = 0; p < SC::NP; p++)
#pragma unroll
            for (int r = 0; r < SC::EPT; r++)
                tws[p][r] = cf{1.f, 0.f};
        run2_prefetch<L, E, S, 1, (SC::TPT <= 64), TPB>(v, t, rows, tws, lds, nx, x, gn, batch, tb, toff8);
    }
}

// One group: loss and gradient of the transforms in `v`.  With PF the
// next group `gn` is loaded into `nx` during the forward passes; the
// weights are read first, so that their wait does not cover those loads.
template <int L, int E, int WG, int S, bool PF>
__device__ __forceinline__ void loss_grad_group(cf (&v)[1 << E], cf (&nx)[1 << E], const cf* __restrict__ x,
                                                int64_t gn, const float* __restrict__ w,
                                                cf* __restrict__ grad, float* __restrict__ loss,
                                                const cf* __restrict__ rows, int64_t g, int64_t batch, int tb,
                                                int t, unsigned toff8, float scale, cf* lds, float* red)
{
    using SC = Sched<L, E>;
    constexpr int EPT = SC::EPT, TPT = SC::TPT, TPB = WG / TPT;
    constexpr bool WAVE = TPT <= 64;
    float wv[EPT];
    load_weights<L, E, TPB>(wv, w, g, batch, tb, toff8 / 2);
    forward_passes<L, E, S, TPB, PF>(v, t, rows, lds, nx, x, gn, batch, tb, toff8);  // X = A x (before its scale)
    float part = 0.f;
#pragma unroll
    for (int m = 0; m < EPT; m++) {
        const cf y = cscale(v[m], scale);
        part += wv[m] * (y.x * y.x + y.y * y.y);
        v[m] = cscale(y, 2.f * wv[m]);
    }
    if constexpr (TPT > 64) {
        // Per-wave sums go to `red`; one workgroup barrier both publishes
        // them and orders the forward's last exchange reads before the
        // adjoint's first writes (a separate barrier for the sum is not
        // needed).  `red` is next written after this group's adjoint
        // exchanges, long after every reader has read it.
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
            part += __shfl_xor(part, off);
        constexpr int W = TPT / 64;
        if ((t & 63) == 0)
            red[tb * W + (t >> 6)] = part;
        __syncthreads();
        if constexpr (TPB == 1) {
            // every thread stores the same sum to the same word: no branch
            // around the store (one would make later waits allow for it
            // not having been issued, and so cover the stores before it)
            float s = 0.f;
#pragma unroll
            for (int i = 0; i < W; i++)
                s += red[i];
            loss[g] = s;
        } else if (t == 0 && g * TPB + tb < batch) {
            float s = 0.f;
#pragma unroll
            for (int i = 0; i < W; i++)
                s += red[tb * W + i];
            loss[g * TPB + tb] = s;
        }
    } else {
        const float total = transform_sum<TPT>(part);
        if (t == 0 && g * TPB + tb < batch)
            loss[g * TPB + tb] = total;
        if constexpr (TPT > 1)
            lds_sync<WAVE>();  // the forward's last exchange is fully read
    }
    transform_passes<L, E, -S>(v, t, rows, lds);  // A^H g (before its scale)
    store_group<L, E, TPB>(v, grad, g, batch, tb, toff8, scale);
    if constexpr (TPT > 1)
        lds_sync<WAVE>();  // LDS is reused by the next group
}

// Persistent: workgroups walk transform groups, loading the next group's x
// while the current one is processed.
template <int L, int E, int WG, int S>
__global__ __launch_bounds__(WG) void k_fft_loss_grad(const cf* __restrict__ x, const float* __restrict__ w,
                                                      cf* __restrict__ grad, float* __restrict__ loss,
                                                      const cf* __restrict__ rows, int64_t batch, float scale)
{
    using SC = Sched<L, E>;
    constexpr int N = SC::N, EPT = SC::EPT, TPT = SC::TPT, TPB = WG / TPT;
    constexpr int REG = TPT > 1 ? Layout2<L, E>::region() : 1;
    __shared__ cf lds[TPT > 1 ? TPB * REG : 1];
    __shared__ float red[TPT > 64 ? TPB * (TPT / 64) : 1];
    const int tid = threadIdx.x, tb = tid / TPT, t = tid % TPT;
    cf* my = lds + (TPT > 1 ? tb * REG : 0);
    const unsigned toff8 = (unsigned)(tb * N + t) * 8u;
    const int64_t ngroups = (batch + TPB - 1) / TPB;
    int64_t g = blockIdx.x;
    if (g >= ngroups)
        return;
    const int64_t stride = gridDim.x;
    cf a[EPT], b[EPT];
    load_group<L, E, TPB>(a, x, g, batch, tb, toff8);
    // `left` groups follow the current one.  Inside the loop the next
    // group's load is unconditional (a conditional one makes the wait
    // before the current group's first use cover the prefetch too) and
    // spread over the forward passes.
    int64_t left = (ngroups - 1 - g) / stride;
#define LG(PF, V, NX, GN) loss_grad_group<L, E, WG, S, PF>(V, NX, x, GN, w, grad, loss, rows, g, batch, tb, t, toff8, scale, my, red)
    while (left >= 2) {
        LG(true, a, b, g + stride);
        g += stride;
        LG(true, b, a, g + stride);
        g += stride;
        left -= 2;
    }
    if (left == 1) {
        LG(true, a, b, g + stride);
        g += stride;
        LG(false, b, a, 0);
    } else {
        LG(false, a, b, 0);
    }
#undef LG
}

template <int L, int E, int WG, int S>
hipError_t launch_loss_grad(const void* x, const float* w, void* grad, float* loss, const void* rows,
                            int64_t batch, float scale, int64_t grid_limit, hipStream_t stream)
{
    constexpr int TPB = WG / Sched<L, E>::TPT;
    int64_t grid = (batch + TPB - 1) / TPB;
    if (grid_limit > 0 && grid > grid_limit)
        grid = grid_limit;
    return launch_kernel((k_fft_loss_grad<L, E, WG, S>), dim3((unsigned)grid), dim3(WG), 0, stream,
                       static_cast<const cf*>(x), w, static_cast<cf*>(grad), loss, static_cast<const cf*>(rows),
                       batch, scale);
}

template <int L, int E, int WG, int S>
int occupancy_loss_grad()
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_fft_loss_grad<L, E, WG, S>, WG, 0) != hipSuccess)
        return 0;
    return blocks;
}

// Menu: EPT 2 only for N <= 4, a whole transform per thread only for
// N <= 16, at most WG threads per transform, LDS <= 64 KiB.
template <int L, int E, int WG>
constexpr bool valid_fused()
{
    if constexpr (E > L || E < 1 || E > 4) {
        return false;
    } else {
        constexpr int TPT = (1 << L) >> E;
        if constexpr (TPT > WG || (E < 2 && L > 2) || (TPT == 1 && L > 4))
            return false;
        else if constexpr (TPT == 1)
            return true;
        else
            return (WG / TPT) * Layout2<L, E>::region() * 8 <= 65536;
    }
}

template <int L, int E, int WG, int S>
void add_fused()
{
    if constexpr (valid_fused<L, E, WG>()) {
        constexpr int TPT = (1 << L) >> E;
        register_loss_grad(KernelLossGrad{L, E, WG, S, &launch_loss_grad<L, E, WG, S>,
                                          &occupancy_loss_grad<L, E, WG, S>,
                                          TPT > 1 ? Layout2<L, E>::rows_total() : 0});
    }
}

template <int L, int E>
void add_fused_wgs()
{
    add_fused<L, E, 64, -1>();
    add_fused<L, E, 64, +1>();
    add_fused<L, E, 128, -1>();
    add_fused<L, E, 128, +1>();
    add_fused<L, E, 256, -1>();
    add_fused<L, E, 256, +1>();
}

struct FusedRegistrar {
    FusedRegistrar()
    {
        add_fused_wgs<MIFFT_LOG2N, 1>();
        add_fused_wgs<MIFFT_LOG2N, 2>();
        add_fused_wgs<MIFFT_LOG2N, 3>();
        add_fused_wgs<MIFFT_LOG2N, 4>();
    }
};
FusedRegistrar fused_registrar;

}  // namespace
}  // namespace mifft
