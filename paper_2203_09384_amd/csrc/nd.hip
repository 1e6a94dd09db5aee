// Axis passes of multidimensional transforms (FP32), in place.
//
// The multidimensional DFT of a d-dimensional array,
//   X[k] = sum_n x[n] prod_a w_{N_a}^{k_a n_a},
// has a kernel that factors over the axes, so it is the 1D transform of
// Eq. (dft) applied along each axis in turn.  The last (contiguous) axis
// runs through the batched 1D kernels; every other axis runs here: a
// transform along an axis of stride s has its points s elements apart, and
// a workgroup takes a tile of TILE transforms adjacent in memory, so that
// row n of the tile is TILE consecutive complex values (one 128-byte line
// when TILE = 16).  Each transform runs the Stockham passes with its own
// LDS region, and the result is written over the input.
#include "device_fft.hpp"
#include "nd.hpp"
#include "tile_fft.hpp"

namespace mifft {
namespace {

// log2 EPT of an axis transform of length 2^L: the whole transform in one
// thread for N <= 4, else as the four-step inner transforms.
constexpr int axis_e(int L) { return L <= 2 ? L : inner_e(L); }
// Transforms per workgroup: 16 (whole 128-byte lines) while 16 transforms
// fit in LDS, 8 for 2048 points.  (Tiles of 8 at 1024 points and 4 at 2048,
// two workgroups per CU, measured 2% faster and 30% slower on MI355X.)
constexpr int axis_tile(int L) { return L <= 10 ? 16 : 8; }
// Long transforms load and store straight between HBM and registers (the
// tile's transform index is the fastest lane index, so each wavefront
// access covers whole rows of the tile); short ones stage the tile through
// LDS so that their exchanges stay inside one wavefront.  Measured on
// MI355X: direct 20% faster per pass at 1024 and 2048 points, equal at 256,
// 4% slower at 128.
constexpr bool axis_direct(int L) { return L >= 9; }

template <int L>
constexpr int axis_wg()
{
    return axis_tile(L) * ((1 << L) >> axis_e(L));
}

template <int L, int E>
__device__ __forceinline__ void unit_rows(TwRegs<L, E>& tws)
{
#pragma unroll
    for (int p = 0; p < Sched<L, E>::NP; p++)
#pragma unroll
        for (int r = 0; r < (1 << E); r++)
            tws[p][r] = cf{1.f, 0.f};
}

// Long transforms: thread (t, c) = tid = t TILE + c holds points t + m TPT
// of tile transform c, so for each m a wavefront reads / writes 64 / TILE
// rows of TILE consecutive complex values straight from / to HBM; LDS only
// carries the Stockham exchanges.  All loads precede the first exchange
// barrier, so the in-place stores are safe.
template <int L, int S>
__device__ __forceinline__ void axis_tile_direct(cf* __restrict__ io, const cf* __restrict__ rows, cf* lds,
                                                 int64_t q0, int64_t count, int log2s, float scale)
{
    constexpr int E = axis_e(L), TILE = axis_tile(L), LT = TILE == 16 ? 4 : 3;
    constexpr int N = 1 << L, EPT = 1 << E, TPT = N / EPT, ST = stage_stride<L, E>();
    constexpr bool WAVE = TPT * TILE <= 64;
    const int tid = threadIdx.x, c = tid & (TILE - 1), t = tid >> LT;
    const int64_t q = q0 + c;
    const bool live = q < count;
    const int64_t base = ((q >> log2s) << (L + log2s)) + (q & ((int64_t(1) << log2s) - 1));
    cf v[EPT];
#pragma unroll
    for (int m = 0; m < EPT; m++)
        v[m] = live ? io[base + ((int64_t)(t + m * TPT) << log2s)] : cf{0.f, 0.f};
    TwRegs<L, E> tws;
    unit_rows<L, E>(tws);
    run2<L, E, S, 1, WAVE>(v, t, rows, tws, lds + c * ST);
    if (live) {
#pragma unroll
        for (int m = 0; m < EPT; m++)
            io[base + ((int64_t)(t + m * TPT) << log2s)] = cscale(v[m], scale);
    }
}

// Short transforms: the tile is staged through LDS (rows of TILE values in,
// one transform per TPT consecutive threads), so each transform's exchanges
// stay inside one wavefront; staged back the same way.
template <int L, int S>
__device__ __forceinline__ void axis_tile_staged(cf* __restrict__ io, const cf* __restrict__ rows, cf* lds,
                                                 int64_t q0, int64_t count, int log2s, float scale)
{
    constexpr int E = axis_e(L), TILE = axis_tile(L), LT = TILE == 16 ? 4 : 3;
    constexpr int N = 1 << L, EPT = 1 << E, TPT = N / EPT, ST = stage_stride<L, E>(), WG = TILE * TPT;
    constexpr bool WAVE = TPT <= 64;
    const int tid = threadIdx.x;
    const int64_t smask = (int64_t(1) << log2s) - 1;
    // element n of tile transform c
    auto addr = [&](int c, int n) -> int64_t {
        const int64_t q = q0 + c;
        return ((q >> log2s) << (L + log2s)) + ((int64_t)n << log2s) + (q & smask);
    };
#pragma unroll
    for (int i = 0; i < TILE * N / WG; i++) {
        const int idx = tid + i * WG;
        const int c = idx & (TILE - 1), n = idx >> LT;
        if (q0 + c < count)
            lds[c * ST + n] = io[addr(c, n)];
    }
    __syncthreads();
    const int tb = tid / TPT, t = tid % TPT;
    cf* my = lds + tb * ST;
    cf v[EPT];
#pragma unroll
    for (int m = 0; m < EPT; m++)
        v[m] = my[t + m * TPT];
    TwRegs<L, E> tws;
    unit_rows<L, E>(tws);
    run2<L, E, S, 1, WAVE>(v, t, rows, tws, my);
    if constexpr (TPT > 1)
        lds_sync<WAVE>();  // the last exchange is fully read
#pragma unroll
    for (int m = 0; m < EPT; m++)
        my[t + m * TPT] = cscale(v[m], scale);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < TILE * N / WG; i++) {
        const int idx = tid + i * WG;
        const int c = idx & (TILE - 1), n = idx >> LT;
        if (q0 + c < count)
            io[addr(c, n)] = lds[c * ST + n];
    }
}

template <int L, int S>
__global__ __launch_bounds__(axis_wg<L>()) void k_axis(cf* __restrict__ io, const cf* __restrict__ rows,
                                                        int64_t count, int log2s, float scale)
{
    constexpr int TILE = axis_tile(L);
    __shared__ cf lds[TILE * stage_stride<L, axis_e(L)>()];
    int64_t tile = blockIdx.x;
    if constexpr (TILE < 16) {
        // The G = 16 / TILE tiles G i .. G i + G-1 share 128-byte lines (when
        // the stride is >= 16): run them on the same XCD (blocks b, b + 8,
        // ... of a chunk of 8 G blocks).
        constexpr int G = 16 / TILE;
        const int64_t b = blockIdx.x;
        tile = (b & ~int64_t(8 * G - 1)) + G * (b & 7) + ((b >> 3) & (G - 1));
    }
    const int64_t q0 = tile * TILE;
    if (q0 >= count)
        return;
    if constexpr (axis_direct(L))
        axis_tile_direct<L, S>(io, rows, lds, q0, count, log2s, scale);
    else
        axis_tile_staged<L, S>(io, rows, lds, q0, count, log2s, scale);
}

template <int L, int S>
hipError_t launch_axis(void* io, const void* rows, int64_t count, int log2s, float scale, hipStream_t stream)
{
    constexpr int TILE = axis_tile(L);
    int64_t grid = (count + TILE - 1) / TILE;
    if (TILE < 16)
        grid = (grid + 127) & ~int64_t(127);  // whole chunks for the XCD grouping
    hipLaunchKernelGGL((k_axis<L, S>), dim3((unsigned)grid), dim3(axis_wg<L>()), 0, stream, static_cast<cf*>(io),
                       static_cast<const cf*>(rows), count, log2s, scale);
    return hipGetLastError();
}

template <int L>
void add_axis()
{
    constexpr int E = axis_e(L);
    const int rows = ((1 << L) >> E) > 1 ? Layout2<L, E>::rows_total() : 0;
    const int lds = (int)(axis_tile(L) * stage_stride<L, E>() * sizeof(cf));
    register_axis(KernelAxis{L, E, -1, axis_tile(L), &launch_axis<L, -1>, rows, lds});
    register_axis(KernelAxis{L, E, +1, axis_tile(L), &launch_axis<L, +1>, rows, lds});
}

struct AxisRegistrar {
    AxisRegistrar()
    {
        add_axis<1>();
        add_axis<2>();
        add_axis<3>();
        add_axis<4>();
        add_axis<5>();
        add_axis<6>();
        add_axis<7>();
        add_axis<8>();
        add_axis<9>();
        add_axis<10>();
        add_axis<11>();
    }
};
AxisRegistrar axis_registrar;

}  // namespace
}  // namespace mifft
