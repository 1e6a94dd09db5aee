// Shapes shared by the kernels that stage tiles of transforms through LDS
// (four-step passes and the axis passes of multidimensional plans): 16
// transforms adjacent in memory per workgroup, each transform inside one
// wavefront, staged with a per-transform LDS stride that spreads the tile
// over the 64 banks.
#pragma once

#include "device_fft.hpp"

namespace mifft {

// log2 EPT of an inner transform of length 2^Li: 16 threads per transform
// up to 256 points, then 16 points per thread (at most 64 threads).
constexpr int inner_e(int Li) { return Li <= 6 ? 2 : (Li == 7 ? 3 : 4); }

// Staging stride (complex elements) of one transform's LDS region: the
// padded Stockham region rounded up to 4 (mod 32), which spreads the 16
// transforms of a tile over distinct banks when the tile is staged.
template <int Li, int Ei>
constexpr int stage_stride()
{
    const int reg = Layout2<Li, Ei>::region();
    const int r = reg % 32;
    return reg + ((4 - r + 32) % 32);
}

}  // namespace mifft
