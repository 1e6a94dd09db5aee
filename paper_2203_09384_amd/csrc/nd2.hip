// Single-pass 2D transforms of arrays that fit one workgroup's LDS
// (N0 x N1 <= 16384 points): one HBM pass instead of one per axis.
//
// The 2D DFT factors into row DFTs then column DFTs (its kernel is a
// product over the axes).  A workgroup holds AP whole arrays; all of an
// array's points are in registers at once (N / EPT threads, EPT points
// each):
//   rows     thread (r, t) loads points t + m TPT1 of row r straight from
//            HBM, runs the Stockham passes with row r's own LDS region for
//            the exchanges (the rows' threads share a wavefront);
//   turn     every row result is written to LDS transposed: column c is
//            contiguous at stride RS0, so it can serve as column c's
//            exchange region;
//   columns  thread (c, t0), c the fastest lane index, reads points
//            t0 + m TPT0 of column c, runs the passes (workgroup barriers:
//            a column's threads span wavefronts) and stores X[n0][c]
//            straight to HBM: consecutive lanes, consecutive addresses.
#include "device_fft.hpp"
#include "launch.hpp"
#include "nd2.hpp"
#include "nd_maps.hpp"

#include <utility>

namespace mifft {
namespace {

template <int L0, int L1>
struct Nd2Shape {
    static constexpr ndm::Nd2Geom G = ndm::nd2_geom(L0, L1);
    static constexpr int E = G.E, EPT = 1 << E;
    static constexpr int N0 = G.N0, N1 = G.N1, N = N0 * N1;
    static constexpr int TPA = G.TPA;  // threads per array
    static constexpr int AP = G.AP;    // arrays per workgroup
    static constexpr int WG = G.WG;
    static constexpr int TPT1 = G.TPT1, TPT0 = G.TPT0;
    static constexpr int RS1 = G.RS1;  // row stride (row phase): the row's exchange region
    static constexpr int RS0 = G.RS0;  // column stride (column phase): odd, for the banks
    static constexpr int ASZ = G.ASZ;  // LDS per array
    static constexpr int LDS = G.LDS;
};

template <int L0, int L1>
constexpr bool nd2_valid()
{
    return ndm::nd2_fits(L0, L1);
}

// Twiddle-row entries (float2) of the column and row transforms as the
// persistent kernel keeps them in LDS: rows padded by ROW_PAD values (see
// load_row).
constexpr int ROW_PAD = 2;

template <int L0, int L1>
struct Nd2Rows {
    using Z = Nd2Shape<L0, L1>;
    static constexpr int R0 = Z::TPT0 > 1 ? padded_rows_total<L0, Z::E, ROW_PAD>() : 0;
    static constexpr int R1 = Z::TPT1 > 1 ? padded_rows_total<L1, Z::E, ROW_PAD>() : 0;
};

// Arrays whose exchanges take more than half of a CU's 160 KiB of LDS run
// one workgroup per CU, which then has nothing to overlap its loads and
// stores with; arrays of one-thread rows (N1 = EPT) load with lanes a whole
// row apart, few requests per cache line, and gain from the overlap too when
// the one-shot grid leaves a CU at most 16 wavefronts.  Those run persistent
// (k_nd2p) when the twiddle rows fit in the LDS left over: as many
// workgroups as are resident at once walk the batch.  (Shapes with longer
// rows at 12-16 wavefronts per CU measured slower persistent: 128 x 64
// 226 -> 256 us, 16 x 256 187 -> 201.)
template <int L0, int L1>
constexpr bool nd2_persistent()
{
    using Z = Nd2Shape<L0, L1>;
    using RW = Nd2Rows<L0, L1>;
    // 1024-point rows excluded: at 1024 threads their registers spill
    // (16 x 1024 measured 280 -> 348 us)
    return Z::AP == 1 && (2 * Z::LDS > 160 * 1024 || (Z::TPT1 == 1 && (160 * 1024 / Z::LDS) * (Z::WG / 64) <= 16)) &&
           Z::LDS + (RW::R0 + RW::R1) * 8 <= 160 * 1024 && Z::EPT % Sched<L0, Z::E>::NP == 0 && L1 < 10;
}

template <int L0, int L1, int S>
__global__ __launch_bounds__((Nd2Shape<L0, L1>::WG)) void k_nd2(const cf* __restrict__ in, cf* __restrict__ out,
                                                             const cf* __restrict__ rows0,
                                                             const cf* __restrict__ rows1, int64_t batch, float scale)
{
    using Z = Nd2Shape<L0, L1>;
    constexpr int E = Z::E, EPT = Z::EPT, N1 = Z::N1, N = Z::N;
    __shared__ cf lds[Z::AP * Z::ASZ];
    const int tid = threadIdx.x, a = tid / Z::TPA, u = tid % Z::TPA;
    const int64_t arr = (int64_t)blockIdx.x * Z::AP + a;
    const bool live = arr < batch;
    cf* my = lds + a * Z::ASZ;
    cf v[EPT];
    TwRegs<L1, E> tw1;
#pragma unroll
    for (int p = 0; p < Sched<L1, E>::NP; p++)
#pragma unroll
        for (int i = 0; i < EPT; i++)
            tw1[p][i] = cf{1.f, 0.f};
    // ---- rows
    {
        const int r = u / Z::TPT1, t = u % Z::TPT1;
        const cf* src = in + arr * N + r * N1;
#pragma unroll
        for (int m = 0; m < EPT; m++)
            v[m] = live ? src[t + m * Z::TPT1] : cf{0.f, 0.f};
        run2<L1, E, S, 1, true>(v, t, rows1, tw1, my + r * Z::RS1);
        __syncthreads();  // every row's exchanges are read
#pragma unroll
        for (int m = 0; m < EPT; m++)
            my[ndm::nd2_turn(r, t + m * Z::TPT1, Z::RS0)] = v[m];
        __syncthreads();
    }
    // ---- columns
    TwRegs<L0, E> tw0;
#pragma unroll
    for (int p = 0; p < Sched<L0, E>::NP; p++)
#pragma unroll
        for (int i = 0; i < EPT; i++)
            tw0[p][i] = cf{1.f, 0.f};
    const int c = u % N1, t0 = u / N1;
    cf* col = my + c * Z::RS0;
#pragma unroll
    for (int m = 0; m < EPT; m++)
        v[m] = col[t0 + m * Z::TPT0];
    if constexpr (Z::TPT0 > 1)
        __syncthreads();  // the column is read before its exchanges overwrite it
    run2<L0, E, S, 1, false>(v, t0, rows0, tw0, col);
    if (live) {
        cf* dst = out + arr * N + c;
#pragma unroll
        for (int m = 0; m < EPT; m++)
            dst[(t0 + m * Z::TPT0) * N1] = cscale(v[m], scale);
    }
}

// Persistent form of k_nd2 for one array per workgroup (nd2_persistent):
// a workgroup walks arrays g = blockIdx.x, + gridDim.x, ... .  While an
// array's column passes run, the next array's row inputs are loaded into the
// row registers (dead after the turn), a slice before each column pass; the
// twiddle rows sit in LDS (padded) for the workgroup's life, so the only global
// loads in the loop are the arrays themselves.  The loop body always
// prefetches; the last array runs after it without (a prefetch under a
// condition would make the wait for the next rows cover the stores too).
template <int L0, int L1, int S>
__global__ __launch_bounds__((Nd2Shape<L0, L1>::WG)) void k_nd2p(const cf* __restrict__ in, cf* __restrict__ out,
                                                              const cf* __restrict__ rows0,
                                                              const cf* __restrict__ rows1, int64_t batch, float scale)
{
    using Z = Nd2Shape<L0, L1>;
    using RW = Nd2Rows<L0, L1>;
    constexpr int E = Z::E, EPT = Z::EPT, N1 = Z::N1, N = Z::N, NP0 = Sched<L0, E>::NP;
    static_assert(Z::AP == 1 && EPT % NP0 == 0, "one array per workgroup, whole slices");
    __shared__ cf lds[Z::ASZ];
    __shared__ cf trow[RW::R0 + RW::R1 > 0 ? RW::R0 + RW::R1 : 1];
    const int tid = threadIdx.x;
    int64_t g = blockIdx.x;
    if (g >= batch)
        return;
    if constexpr (RW::R0 > 0)
        copy_rows_padded<L0, E, ROW_PAD>(trow, rows0, tid, Z::WG);
    if constexpr (RW::R1 > 0)
        copy_rows_padded<L1, E, ROW_PAD>(trow + RW::R0, rows1, tid, Z::WG);
    const cf* tr0 = trow;
    const cf* tr1 = trow + RW::R0;
    TwRegs<L1, E> tw1;
#pragma unroll
    for (int p = 0; p < Sched<L1, E>::NP; p++)
#pragma unroll
        for (int i = 0; i < EPT; i++)
            tw1[p][i] = cf{1.f, 0.f};
    TwRegs<L0, E> tw0;
#pragma unroll
    for (int p = 0; p < NP0; p++)
#pragma unroll
        for (int i = 0; i < EPT; i++)
            tw0[p][i] = cf{1.f, 0.f};
    const int r = tid / Z::TPT1, t = tid % Z::TPT1;  // rows: thread t of row r
    const int c = tid % N1, t0 = tid / N1;           // columns: thread t0 of column c
    const cf* src = in + r * N1 + t;                 // + g N + m TPT1: point t + m TPT1 of row r
    cf* myrow = lds + r * Z::RS1;
    cf* col = lds + c * Z::RS0;
    cf a[EPT], v[EPT];
#pragma unroll
    for (int m = 0; m < EPT; m++)
        a[m] = src[g * N + m * Z::TPT1];
    __syncthreads();  // twiddle rows in place
    // rows, the turn, and the column's points into v
    auto rows_and_turn = [&]() {
        run2<L1, E, S, 1, true, 0, ROW_PAD>(a, t, tr1, tw1, myrow);
        __syncthreads();  // every row's exchanges are read
#pragma unroll
        for (int m = 0; m < EPT; m++)
            lds[ndm::nd2_turn(r, t + m * Z::TPT1, Z::RS0)] = a[m];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < EPT; m++)
            v[m] = col[t0 + m * Z::TPT0];
        if constexpr (Z::TPT0 > 1)
            __syncthreads();  // the column is read before its exchanges overwrite it
    };
    auto store = [&]() {
        cf* dst = out + g * N + c;
#pragma unroll
        for (int m = 0; m < EPT; m++)
            dst[(t0 + m * Z::TPT0) * N1] = cscale(v[m], scale);
    };
    // The loop is rotated (rows of the next array at the end of the body), so
    // the prefetched rows are used in the body that loaded them and the wait
    // for them leaves the stores issued in between in flight.
    const int64_t stride = gridDim.x;
    int64_t left = (batch - 1 - g) / stride;
    rows_and_turn();
    while (left > 0) {
        const cf* nsrc = src + (g + stride) * N;
        auto slice = [&](auto pc) {
            constexpr int P = decltype(pc)::value;
#pragma unroll
            for (int m = P * EPT / NP0; m < (P + 1) * EPT / NP0; m++)
                a[m] = nsrc[m * Z::TPT1];
        };
        run2_slices<L0, E, S, ROW_PAD, NP0>(v, t0, tr0, rows0, col, slice);
        store();
        g += stride;
        --left;
        __syncthreads();  // the column exchanges are read before the next rows use LDS
        rows_and_turn();
    }
    run2<L0, E, S, 1, false, 0, ROW_PAD>(v, t0, tr0, tw0, col);
    store();
}

template <int L0, int L1, int S>
int nd2_slots()
{
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 0;
    if (cached[dev] == 0) {
        int cus = 0, per = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_nd2p<L0, L1, S>, Nd2Shape<L0, L1>::WG, 0) !=
                hipSuccess)
            return 0;
        cached[dev] = cus * per;
    }
    return cached[dev];
}

template <int L0, int L1, int S>
constexpr auto nd2_slots_fn()
{
    if constexpr (nd2_persistent<L0, L1>())
        return &nd2_slots<L0, L1, S>;
    else
        return static_cast<int (*)()>(nullptr);
}

template <int L0, int L1, int S>
hipError_t launch_nd2(const void* in, void* out, const void* rows0, const void* rows1, int64_t batch, float scale,
                      hipStream_t stream)
{
    using Z = Nd2Shape<L0, L1>;
    if constexpr (nd2_persistent<L0, L1>()) {
        const int slots = nd2_slots<L0, L1, S>();
        if (slots > 0) {
            const int64_t grid = batch > slots ? slots : batch;
            return launch_kernel((k_nd2p<L0, L1, S>), dim3((unsigned)grid), dim3(Z::WG), 0, stream,
                                 static_cast<const cf*>(in), static_cast<cf*>(out), static_cast<const cf*>(rows0),
                                 static_cast<const cf*>(rows1), batch, scale);
        }
    }
    const int64_t grid = (batch + Z::AP - 1) / Z::AP;
    return launch_kernel((k_nd2<L0, L1, S>), dim3((unsigned)grid), dim3(Z::WG), 0, stream,
                       static_cast<const cf*>(in), static_cast<cf*>(out), static_cast<const cf*>(rows0),
                       static_cast<const cf*>(rows1), batch, scale);
}

template <int L0, int L1>
void add_nd2()
{
    if constexpr (nd2_valid<L0, L1>()) {
        using Z = Nd2Shape<L0, L1>;
        const int r0 = Z::TPT0 > 1 ? Layout2<L0, Z::E>::rows_total() : 0;
        const int r1 = Z::TPT1 > 1 ? Layout2<L1, Z::E>::rows_total() : 0;
        register_nd2(KernelNd2{L0, L1, Z::E, -1, Z::AP, Z::WG, &launch_nd2<L0, L1, -1>, r0, r1, Z::LDS,
                               nd2_slots_fn<L0, L1, -1>()});
        register_nd2(KernelNd2{L0, L1, Z::E, +1, Z::AP, Z::WG, &launch_nd2<L0, L1, +1>, r0, r1, Z::LDS,
                               nd2_slots_fn<L0, L1, +1>()});
    }
}

template <int L0, int... L1s>
void add_row(std::integer_sequence<int, L1s...>)
{
    (add_nd2<L0, L1s + 1>(), ...);
}

template <int... L0s>
void add_all(std::integer_sequence<int, L0s...>)
{
    (add_row<L0s + 1>(std::make_integer_sequence<int, 13>{}), ...);
}

struct Nd2Registrar {
    Nd2Registrar() { add_all(std::make_integer_sequence<int, 13>{}); }
};
Nd2Registrar nd2_registrar;

}  // namespace
}  // namespace mifft
