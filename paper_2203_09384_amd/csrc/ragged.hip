// Persistent kernel for ragged batches (mixed power-of-two lengths packed
// back to back), compiled once per workgroup size (-DMIFFT_RAGGED_WG).
//
// The paper finds that for transforms running O(10) us, kernel dispatch --
// not the transform -- dominates (section "Results", launch-latency table).
// A mixed batch would otherwise need one launch per length.  Here one
// launch covers every tile of the plan (tiles sorted largest length first)
// and each workgroup dispatches, per tile, to the transform instantiated for
// that (length, elements per thread); every such instantiation is the same
// Stockham pass machinery as the batched kernels.
//
// Tiles are dealt to workgroups statically, in rounds of gridDim.x, the
// order reversed every other round (workgroup b takes tile r G + b in even
// rounds r, r G + G - 1 - b in odd ones), so that each workgroup's share of
// the longest-first list is balanced.  A shared atomic counter would balance
// dynamically, but its atomics serialise on one address (about 10 ns each on
// MI355X, which made them most of the launch); the static deal needs no
// device state, so a launch replays from a hipGraph as it is.
#include "device_fft.hpp"
#include "launch.hpp"
#include "ragged_kernel.hpp"

#ifndef MIFFT_RAGGED_WG
#error "compile with -DMIFFT_RAGGED_WG=<64|128|256>"
#endif

namespace mifft {
namespace {

// LDS elements a kernel needs: the largest per-tile region over its pairs.
template <int WG, int MAXE>
constexpr int ragged_lds_elems()
{
    int m = 0;
    for (int L = 1; L <= 11; L++)
        for (int E = 1; E <= 4; E++) {
            if (!ragged_pair_ok(L, E, WG, MAXE))
                continue;
            const int tpt = (1 << L) >> E;
            if (tpt < 2)
                continue;
            const int need = (WG / tpt) * idx::region(L, E);
            m = need > m ? need : m;
        }
    return m > 0 ? m : 1;
}

template <int L, int E, int WG, int S>
__device__ __forceinline__ void ragged_tile(const RaggedArgs& a, const RaggedTile& tile, cf* lds, int tid)
{
    using SC = Sched<L, E>;
    constexpr int N = SC::N, EPT = SC::EPT, TPT = SC::TPT;
    const int tb = tid / TPT, t = tid % TPT;
    const bool live = tb < tile.count;
    const int64_t off = live ? a.toff[tile.first + tb] : 0;
    const cf* __restrict__ src = static_cast<const cf*>(a.in) + off;
    cf* __restrict__ dst = static_cast<cf*>(a.out) + off;
    const float scale = a.inv ? 1.0f / (float)N : 1.0f;
    cf v[EPT];
#pragma unroll
    for (int m = 0; m < EPT; m++)
        v[m] = live ? src[t + m * TPT] : cf{0.f, 0.f};
    TwRegs<L, E> tws;
#pragma unroll
    for (int p = 0; p < SC::NP; p++)
#pragma unroll
        for (int r = 0; r < EPT; r++)
            tws[p][r] = cf{1.f, 0.f};
    if constexpr (TPT == 1) {
        pass_compute2<L, E, S, 0>(v, tws[0]);
    } else {
        constexpr int REG = Layout2<L, E>::region();
        run2<L, E, S, 1, (TPT <= 64)>(v, t, static_cast<const cf*>(a.rows) + a.rows_off[L], tws,
                                      lds + tb * REG);
    }
    if (live) {
#pragma unroll
        for (int m = 0; m < EPT; m++)
            dst[t + m * TPT] = cscale(v[m], scale);
    }
}

#define MIFFT_RCASE(L, E)                                      \
    case (L) * 8 + (E):                                        \
        if constexpr (ragged_pair_ok(L, E, WG, MAXE))          \
            ragged_tile<L, E, WG, S>(a, tile, lds, tid);       \
        break;

template <int WG, int MAXE, int S>
__global__ __launch_bounds__(WG) void k_fft_ragged(RaggedArgs a)
{
    __shared__ cf lds[ragged_lds_elems<WG, MAXE>()];
    const int G = gridDim.x, b = blockIdx.x;
    for (int base = 0, round = 0; base < a.ntiles; base += G, round++) {
        const int ti = base + ((round & 1) ? G - 1 - b : b);
        if (ti >= a.ntiles)
            break;  // only in the last round
        if (round > 0)
            __syncthreads();  // the previous tile's LDS use is over
        const RaggedTile tile = a.tiles[ti];
        // The thread index is made opaque per tile: otherwise the address
        // arithmetic of every case is hoisted out of the loop and stays
        // live across all of them (294 VGPRs, one wavefront per SIMD,
        // instead of the largest single case's 83).
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        switch (tile.log2n * 8 + tile.log2e) {
            MIFFT_RCASE(1, 1)
            MIFFT_RCASE(2, 1) MIFFT_RCASE(2, 2)
            MIFFT_RCASE(3, 2) MIFFT_RCASE(3, 3)
            MIFFT_RCASE(4, 2) MIFFT_RCASE(4, 3) MIFFT_RCASE(4, 4)
            MIFFT_RCASE(5, 2) MIFFT_RCASE(5, 3) MIFFT_RCASE(5, 4)
            MIFFT_RCASE(6, 2) MIFFT_RCASE(6, 3) MIFFT_RCASE(6, 4)
            MIFFT_RCASE(7, 2) MIFFT_RCASE(7, 3) MIFFT_RCASE(7, 4)
            MIFFT_RCASE(8, 2) MIFFT_RCASE(8, 3) MIFFT_RCASE(8, 4)
            MIFFT_RCASE(9, 2) MIFFT_RCASE(9, 3) MIFFT_RCASE(9, 4)
            MIFFT_RCASE(10, 2) MIFFT_RCASE(10, 3) MIFFT_RCASE(10, 4)
            MIFFT_RCASE(11, 2) MIFFT_RCASE(11, 3) MIFFT_RCASE(11, 4)
            default:
                break;
        }
    }
}

#undef MIFFT_RCASE

template <int WG, int MAXE, int S>
hipError_t launch_ragged(const RaggedArgs& a, int grid, hipStream_t stream)
{
    return launch_kernel((k_fft_ragged<WG, MAXE, S>), dim3(grid), dim3(WG), 0, stream, a);
}

template <int WG, int MAXE, int S>
int occupancy_ragged()
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_fft_ragged<WG, MAXE, S>, WG, 0) != hipSuccess)
        return 0;
    return blocks;
}

template <int WG, int MAXE, int S>
void add_ragged()
{
    register_ragged(KernelRagged{WG, MAXE, S, &launch_ragged<WG, MAXE, S>, &occupancy_ragged<WG, MAXE, S>,
                                 (int)(ragged_lds_elems<WG, MAXE>() * sizeof(cf))});
}

struct RaggedRegistrar {
    RaggedRegistrar()
    {
        add_ragged<MIFFT_RAGGED_WG, 3, -1>();
        add_ragged<MIFFT_RAGGED_WG, 3, +1>();
        add_ragged<MIFFT_RAGGED_WG, 4, -1>();
        add_ragged<MIFFT_RAGGED_WG, 4, +1>();
    }
};
RaggedRegistrar ragged_registrar;

}  // namespace
}  // namespace mifft
