// Tiles of transforms adjacent in memory, one tile per workgroup: shapes and
// tile bodies shared by the four-step passes and the axis passes of
// multidimensional plans.  Each transform has its own LDS region, at a
// stride that spreads the tile over the 64 banks.
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

// ---------------------------------------------------------------- axis tiles
// A tile is TILE transforms of length 2^L along an axis of stride 2^log2s,
// adjacent in memory: transform q starts at element
// (q >> log2s) 2^(L + log2s) + (q & (2^log2s - 1)), its point n is 2^log2s
// elements further per n, so row n of a tile is TILE consecutive values
// when the stride is at least TILE.  Used in place.

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
    const int64_t base = idx::axis_elem(q, 0, L, log2s);
    cf v[EPT];
#pragma unroll
    for (int m = 0; m < EPT; m++)
        v[m] = live ? ld_c(io + base + ((int64_t)(t + m * TPT) << log2s)) : cf{0.f, 0.f};
    TwRegs<L, E> tws;
    unit_rows<L, E>(tws);
    run2<L, E, S, 1, WAVE>(v, t, rows, tws, lds + c * ST);
    if (live) {
#pragma unroll
        for (int m = 0; m < EPT; m++)
            st_c(io + base + ((int64_t)(t + m * TPT) << log2s), cscale(v[m], scale));
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
    // element n of tile transform c
    auto addr = [&](int c, int n) -> int64_t { return idx::axis_elem(q0 + c, n, L, log2s); };
#pragma unroll
    for (int i = 0; i < TILE * N / WG; i++) {
        const int idx = tid + i * WG;
        const int c = idx & (TILE - 1), n = idx >> LT;
        if (q0 + c < count)
            lds[c * ST + n] = ld_c(io + addr(c, n));
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
            st_c(io + addr(c, n), lds[c * ST + n]);
    }
}

}  // namespace mifft
