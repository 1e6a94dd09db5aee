// Lengths 2^12 .. 2^20 (FP32): four-step Cooley-Tukey split N = N1 * N2.
//
// With n = n1 N2 + n2 and k = k1 + N1 k2 the DFT of Eq. (dft) factors as
//   X[k1 + N1 k2] = sum_n2 w_N2^{n2 k2} ( w_N^{n2 k1} sum_n1 x[n1 N2 + n2] w_N1^{n1 k1} )
// i.e. the radix-N1 / radix-N2 Cooley-Tukey split of Eq. (radix2) taken
// once with large radices.  Two kernels:
//   pass 1  column DFTs of length N1 (stride N2) times w_N^{n2 k1}, stored
//           to Y[k1 + N1 n2] of `out` (so pass 2's tile is read and written
//           in place);
//   pass 2  row DFTs of length N2 over n2, in place in `out`, output
//           X[k1 + N1 k2] (times the plan's scale).
// Each workgroup owns a tile of 16 transforms (16 columns, or 16 rows k1)
// so that every global load and store is a run of 16 complex values (one
// 128-byte line); the tile is staged through LDS, transformed with the same
// Stockham passes as the batched kernels (each transform inside one
// wavefront) and staged back for the store.  w_N^j is built from a two-level
// FP32 table (w_N^{1024 a} and w_N^{b}, both from FP64 sincospi).
#include "device_fft.hpp"
#include "fourstep.hpp"
#include "tile_fft.hpp"

namespace mifft {
namespace {

constexpr int TILE = 16;

template <int S>
__device__ __forceinline__ cf big_twiddle(const cf* __restrict__ lo, const cf* __restrict__ hi, unsigned j)
{
    cf w = cmul(hi[j >> 10], lo[j & 1023u]);
    if constexpr (S > 0)
        w.y = -w.y;
    return w;
}

// Pass 1: tile = columns n2 in [16 nb, 16 nb + 16) of transform b.
template <int L1, int L2, int S>
__global__ __launch_bounds__(TILE*((1 << L1) >> inner_e(L1))) void k_fourstep1(
    const cf* __restrict__ in, cf* __restrict__ out, const cf* __restrict__ rows, const cf* __restrict__ tlo,
    const cf* __restrict__ thi)
{
    constexpr int E = inner_e(L1), N1 = 1 << L1, N2 = 1 << L2, N = N1 * N2;
    constexpr int EPT = 1 << E, TPT = N1 / EPT, WG = TILE * TPT, ST = stage_stride<L1, E>();
    __shared__ cf lds[TILE * ST];
    const int tid = threadIdx.x;
    const int64_t b = blockIdx.x / (N2 / TILE);
    const int nb = blockIdx.x % (N2 / TILE);
    const cf* src = in + b * N + nb * TILE;
    // stage: 16 consecutive columns per row n1 (one 128-byte line)
#pragma unroll
    for (int i = 0; i < TILE * N1 / WG; i++) {
        const int idx = tid + i * WG;
        const int c = idx & (TILE - 1), n1 = idx >> 4;
        lds[c * ST + n1] = src[(int64_t)n1 * N2 + c];
    }
    __syncthreads();
    const int tb = tid / TPT, t = tid % TPT;
    cf* my = lds + tb * ST;
    cf v[EPT];
#pragma unroll
    for (int m = 0; m < EPT; m++)
        v[m] = my[t + m * TPT];
    TwRegs<L1, E> tws;
#pragma unroll
    for (int p = 0; p < Sched<L1, E>::NP; p++)
#pragma unroll
        for (int r = 0; r < EPT; r++)
            tws[p][r] = cf{1.f, 0.f};
    run2<L1, E, S, 1, true>(v, t, rows, tws, my);  // transform tb lives in one wavefront
    const unsigned n2 = nb * TILE + tb;
#pragma unroll
    for (int m = 0; m < EPT; m++) {
        const unsigned k1 = t + m * TPT;
        v[m] = cmul(v[m], big_twiddle<S>(tlo, thi, n2 * k1));
    }
    lds_sync<true>();  // this wavefront's last exchange is read
#pragma unroll
    for (int m = 0; m < EPT; m++)
        my[t + m * TPT] = v[m];
    __syncthreads();
    // the tile's outputs Y[k1 + N1 n2] form one contiguous block
    cf* dst = out + b * N + (int64_t)nb * TILE * N1;
#pragma unroll
    for (int i = 0; i < TILE * N1 / WG; i++) {
        const int idx = tid + i * WG;
        const int c = idx / N1, k1 = idx % N1;
        dst[idx] = lds[c * ST + k1];
    }
}

// Pass 2 (in place): tile = rows k1 in [16 kb, 16 kb + 16) of transform b,
// elements Y[k1 + N1 n2]; outputs X[k1 + N1 k2] at the same addresses.
template <int L1, int L2, int S>
__global__ __launch_bounds__(TILE*((1 << L2) >> inner_e(L2))) void k_fourstep2(cf* __restrict__ io,
                                                                              const cf* __restrict__ rows,
                                                                              float scale)
{
    constexpr int E = inner_e(L2), N1 = 1 << L1, N2 = 1 << L2, N = N1 * N2;
    constexpr int EPT = 1 << E, TPT = N2 / EPT, WG = TILE * TPT, ST = stage_stride<L2, E>();
    __shared__ cf lds[TILE * ST];
    const int tid = threadIdx.x;
    const int64_t b = blockIdx.x / (N1 / TILE);
    const int kb = blockIdx.x % (N1 / TILE);
    cf* base = io + b * N + kb * TILE;
#pragma unroll
    for (int i = 0; i < TILE * N2 / WG; i++) {
        const int idx = tid + i * WG;
        const int c = idx & (TILE - 1), n2 = idx >> 4;
        lds[c * ST + n2] = base[(int64_t)n2 * N1 + c];
    }
    __syncthreads();
    const int tb = tid / TPT, t = tid % TPT;
    cf* my = lds + tb * ST;
    cf v[EPT];
#pragma unroll
    for (int m = 0; m < EPT; m++)
        v[m] = my[t + m * TPT];
    TwRegs<L2, E> tws;
#pragma unroll
    for (int p = 0; p < Sched<L2, E>::NP; p++)
#pragma unroll
        for (int r = 0; r < EPT; r++)
            tws[p][r] = cf{1.f, 0.f};
    run2<L2, E, S, 1, true>(v, t, rows, tws, my);
    lds_sync<true>();
#pragma unroll
    for (int m = 0; m < EPT; m++)
        my[t + m * TPT] = cscale(v[m], scale);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < TILE * N2 / WG; i++) {
        const int idx = tid + i * WG;
        const int c = idx & (TILE - 1), k2 = idx >> 4;
        base[(int64_t)k2 * N1 + c] = lds[c * ST + k2];
    }
}

template <int L1, int L2, int S>
hipError_t launch_fourstep(const void* in, void* out, const void* rows1, const void* rows2, const void* tlo,
                           const void* thi, int64_t batch, float scale, hipStream_t stream)
{
    constexpr int WG1 = TILE * ((1 << L1) >> inner_e(L1));
    constexpr int WG2 = TILE * ((1 << L2) >> inner_e(L2));
    const int64_t g1 = batch * ((1 << L2) / TILE), g2 = batch * ((1 << L1) / TILE);
    hipLaunchKernelGGL((k_fourstep1<L1, L2, S>), dim3((unsigned)g1), dim3(WG1), 0, stream,
                       static_cast<const cf*>(in), static_cast<cf*>(out), static_cast<const cf*>(rows1),
                       static_cast<const cf*>(tlo), static_cast<const cf*>(thi));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL((k_fourstep2<L1, L2, S>), dim3((unsigned)g2), dim3(WG2), 0, stream, static_cast<cf*>(out),
                       static_cast<const cf*>(rows2), scale);
    return hipGetLastError();
}

template <int L>
void add_len()
{
    constexpr int L1 = (L + 1) / 2, L2 = L / 2;
    const FourStep fs{L, L1, L2, inner_e(L1), inner_e(L2), Layout2<L1, inner_e(L1)>::rows_total(),
                      Layout2<L2, inner_e(L2)>::rows_total(), &launch_fourstep<L1, L2, -1>,
                      &launch_fourstep<L1, L2, +1>,
                      (int)(TILE * stage_stride<L1, inner_e(L1)>() * sizeof(cf)),
                      (int)(TILE * stage_stride<L2, inner_e(L2)>() * sizeof(cf))};
    register_fourstep(fs);
}

struct FourStepRegistrar {
    FourStepRegistrar()
    {
        add_len<12>();
        add_len<13>();
        add_len<14>();
        add_len<15>();
        add_len<16>();
        add_len<17>();
        add_len<18>();
        add_len<19>();
        add_len<20>();
    }
};
FourStepRegistrar fourstep_registrar;

}  // namespace

// Two-level twiddles of length N = 2^L: lo[b] = w_N^b (b < 1024),
// hi[a] = w_N^{1024 a} (a < N / 1024), w_N = exp(-2 pi i / N), FP64 sincospi
// rounded once to FP32.
__global__ void k_twiddle_big(float2* __restrict__ lo, float2* __restrict__ hi, int L)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int nhi = 1 << (L - 10);
    if (i >= 1024 + nhi)
        return;
    const int64_t j = i < 1024 ? i : (int64_t)(i - 1024) << 10;
    double s, c;
    sincospi(2.0 * (double)j / (double)(int64_t(1) << L), &s, &c);
    const float2 w = float2{(float)c, (float)(-s)};
    if (i < 1024)
        lo[i] = w;
    else
        hi[i - 1024] = w;
}

hipError_t launch_twiddle_big(void* lo, void* hi, int L, hipStream_t stream)
{
    const int total = 1024 + (1 << (L - 10));
    hipLaunchKernelGGL(k_twiddle_big, dim3((total + 255) / 256), dim3(256), 0, stream, static_cast<float2*>(lo),
                       static_cast<float2*>(hi), L);
    return hipGetLastError();
}

}  // namespace mifft
