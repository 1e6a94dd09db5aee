// Ragged batches of mixed power-of-two lengths: types shared by the
// persistent kernel (ragged.hip) and its planner (ragged_plan.cpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mifft {

// One unit of work: `count` transforms of length 2^log2n, all processed by
// one workgroup pass with 2^log2e elements per thread; their element
// offsets are toff[first .. first + count).
struct RaggedTile {
    int log2n, log2e, count, first;
};

struct RaggedArgs {
    const void* in;
    void* out;
    const void* rows;           // concatenated per-length twiddle rows
    const int64_t* toff;        // element offset of each transform, tile order
    const RaggedTile* tiles;    // largest lengths first
    int ntiles;
    int inv;                    // nonzero: scale each transform by 1/its length
    int rows_off[12];           // start of length 2^L's rows in `rows`
};

using LaunchRagged = hipError_t (*)(const RaggedArgs& a, int grid, hipStream_t stream);

struct KernelRagged {
    int wg, maxe, sign;
    LaunchRagged fn;
    int (*occupancy)();
    int lds_bytes;
};

void register_ragged(const KernelRagged& k);
const KernelRagged* find_ragged(int wg, int maxe, int sign);

// Which (log2 N, log2 EPT) pairs a ragged kernel with workgroup size WG and
// largest log2 EPT MAXE contains: EPT <= N, at most WG threads per
// transform, EPT = 2 only for N <= 4.
constexpr bool ragged_pair_ok(int L, int E, int WG, int MAXE)
{
    return L >= 1 && L <= 11 && E >= 1 && E <= MAXE && E <= L && (E >= 2 || L <= 2) &&
           ((1 << L) >> E) <= WG;
}

}  // namespace mifft
