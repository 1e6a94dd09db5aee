// Tiles of transforms adjacent in memory, one tile per workgroup: shapes and
// tile bodies shared by the four-step passes and the axis passes of
// multidimensional plans.  Each transform has its own LDS region, at a
// stride that spreads the tile over the 64 banks.
#pragma once

#include "device_fft.hpp"
#include "launch.hpp"

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

// Kernels in this header are per translation unit (anonymous namespace),
// like every kernel of the library.
namespace {

// Axis passes whose tile fills more than half of a CU's LDS (1024-point
// axes: one 1024-thread workgroup per CU, which a workgroup per tile leaves
// nothing to overlap with) run persistent when every tile is whole: a workgroup walks the tiles in the one-shot grid's order (rounds
// of gridDim.x workgroups, so the XCD grouping of tiles sharing lines
// holds), loading its next tile into a second register set a slice before
// each pass.  The twiddle rows sit in LDS, padded, for the workgroup's
// life.  The prefetched tile is waited for only after the current tile's
// stores, which stay in flight.  With every tile whole no load or store is
// conditional, and addresses are a uniform tile base plus a 32-bit
// per-thread byte offset.
constexpr int AX_ROW_PAD = 2;

template <int L>
constexpr int axis_lds_bytes()
{
    return axis_tile(L) * stage_stride<L, axis_e(L)>() * 8;
}

// Passes whose twiddle rows sit in LDS beside the tile.
template <int L>
constexpr int axis_lds_row_passes()
{
    return rows_prefix_passes<L, axis_e(L), AX_ROW_PAD>(160 * 1024 - axis_lds_bytes<L>());
}

// All rows must fit: at 2048 points only the first two passes' do, and
// reading the last pass's row from the cache costs the registers the second
// tile needs (128 bytes per lane spilled; 2D 2048 x 2048 459 -> 568 us).
template <int L>
constexpr bool axis_persistent()
{
    return axis_direct(L) && 2 * axis_lds_bytes<L>() > 160 * 1024 &&
           axis_lds_row_passes<L>() == Sched<L, axis_e(L)>::NP;
}

template <int L, int S>
__global__ __launch_bounds__(axis_wg<L>()) void k_axis_p(cf* __restrict__ io, const cf* __restrict__ rows,
                                                          int64_t ntiles, int log2s, float scale)
{
    constexpr int E = axis_e(L), TILE = axis_tile(L), LT = TILE == 16 ? 4 : 3, G = 16 / TILE;
    constexpr int N = 1 << L, EPT = 1 << E, TPT = N / EPT, ST = stage_stride<L, E>(), WG = axis_wg<L>();
    constexpr int NP = Sched<L, E>::NP, K = axis_lds_row_passes<L>();
    __shared__ cf lds[TILE * ST];
    __shared__ cf trow[padded_rows_prefix<L, E, AX_ROW_PAD>(K) > 0 ? padded_rows_prefix<L, E, AX_ROW_PAD>(K) : 1];
    const int tid = threadIdx.x, c = tid & (TILE - 1), t = tid >> LT;
    int64_t vb = blockIdx.x;
    if (vb >= ntiles)
        return;
    copy_rows_prefix_padded<L, E, AX_ROW_PAD, K>(trow, rows, tid, WG);
    cf* my = lds + c * ST;
    const int64_t P = gridDim.x;
    // Point t + m TPT of tile transform c lies c + ((t + m TPT) << log2s)
    // elements past the tile's first element (the stride is at least TILE).
    const unsigned loff = (unsigned)(c + (t << log2s)) * 8u;
    const unsigned step8 = (unsigned)TPT << (log2s + 3);
    auto tbase = [&](int64_t b) {
        return reinterpret_cast<char*>(io + idx::axis_elem(idx::xcd_group_tile(b, G) * TILE, 0, L, log2s));
    };
    cf a[EPT], bb[EPT];
    {
        const char* gb = tbase(vb);
#pragma unroll
        for (int m = 0; m < EPT; m++)
            a[m] = ld_data<false>(gb + (loff + m * step8));
    }
    __syncthreads();  // twiddle rows in place
    auto store = [&](const cf (&v)[EPT], int64_t b) {
        char* gb = tbase(b);
#pragma unroll
        for (int m = 0; m < EPT; m++)
            st_data<false>(gb + (loff + m * step8), cscale(v[m], scale));
    };
    // transform the tile at position b (in v) while loading position b + P into nx
    auto run = [&](cf (&v)[EPT], cf (&nx)[EPT], int64_t b) {
        const char* nb = tbase(b + P);
        auto slice = [&](auto pc) {
            constexpr int Q = decltype(pc)::value;
#pragma unroll
            for (int m = Q * EPT / NP; m < (Q + 1) * EPT / NP; m++)
                nx[m] = ld_data<false>(nb + (loff + m * step8));
        };
        run2_slices<L, E, S, AX_ROW_PAD, K>(v, t, trow, rows, my, slice);
        store(v, b);
        __syncthreads();  // this tile's exchanges are read before the next tile's
    };
    // One body: the prefetched tile is copied into the working set at the
    // body's end, after the stores, so the wait for it there leaves those
    // stores in flight, and the body's code appears once.
    for (int64_t left = (ntiles - 1 - vb) / P; left > 0; --left) {
        run(a, bb, vb);
#pragma unroll
        for (int m = 0; m < EPT; m++)
            a[m] = bb[m];
        vb += P;
    }
    auto none = [](auto) {};
    run2_slices<L, E, S, AX_ROW_PAD, K>(a, t, trow, rows, my, none);
    store(a, vb);
}

inline int axis_cus()
{
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 0;
    if (cached[dev] == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        cached[dev] = cus;
    }
    return cached[dev];
}


// Launches the persistent axis pass when it applies (axis_persistent, every
// tile whole, every chunk of the XCD grouping full, rows of at least TILE
// values so tiles are disjoint columns, and a transform's span addressable
// with 32-bit byte offsets).  Returns false, launching nothing, otherwise.
template <int L, int S>
bool launch_axis_persistent(void* io, const void* rows, int64_t count, int log2s, float scale, hipStream_t stream,
                            hipError_t* err)
{
    if constexpr (!axis_persistent<L>()) {
        return false;
    } else {
        constexpr int TILE = axis_tile(L);
        const int64_t ntiles = count / TILE;
        const int cus = axis_cus();
        const bool span32 = ((int64_t(1) << (L + log2s)) * 8) <= (int64_t(1) << 32);
        if (count % TILE != 0 || ntiles % (128 / TILE) != 0 || log2s < (TILE == 16 ? 4 : 3) || !span32 || cus <= 0)
            return false;
        const int64_t g = ntiles < cus ? ntiles : cus;
        *err = launch_kernel((k_axis_p<L, S>), dim3((unsigned)g), dim3(axis_wg<L>()), 0, stream, static_cast<cf*>(io),
                             static_cast<const cf*>(rows), ntiles, log2s, scale);
        return true;
    }
}

}  // namespace

}  // namespace mifft
