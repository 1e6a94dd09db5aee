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
#include "launch.hpp"
#include "nd.hpp"
#include "tile_fft.hpp"

namespace mifft {
namespace {

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
        tile = idx::xcd_group_tile(b, G);
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
    hipError_t e;
    if (launch_axis_persistent<L, S>(io, rows, count, log2s, scale, stream, &e))
        return e;
    int64_t grid = (count + TILE - 1) / TILE;
    if (TILE < 16)
        grid = (grid + 127) & ~int64_t(127);  // whole chunks for the XCD grouping
    return launch_kernel((k_axis<L, S>), dim3((unsigned)grid), dim3(axis_wg<L>()), 0, stream, static_cast<cf*>(io),
                       static_cast<const cf*>(rows), count, log2s, scale);
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
