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

#include <utility>

namespace mifft {
namespace {

constexpr int nd2_e(int L0, int L1)
{
    const int m = L0 < L1 ? L0 : L1;
    return m < 4 ? m : 4;
}

// Column stride in the transposed layout: the column's Stockham region,
// rounded up to an odd number of complex values so that lanes reading
// consecutive columns spread over the 64 banks.
template <int L0, int E>
constexpr int col_stride()
{
    const int r = Layout2<L0, E>::region();
    return (r & 1) ? r : r + 1;
}

template <int L0, int L1>
struct Nd2Shape {
    static constexpr int E = nd2_e(L0, L1), EPT = 1 << E;
    static constexpr int N0 = 1 << L0, N1 = 1 << L1, N = N0 * N1;
    static constexpr int TPA = N / EPT;                  // threads per array
    static constexpr int AP = TPA >= 256 ? 1 : 256 / TPA;  // arrays per workgroup
    static constexpr int WG = AP * TPA;
    static constexpr int TPT1 = N1 / EPT, TPT0 = N0 / EPT;
    static constexpr int RS1 = Layout2<L1, E>::region();  // row stride (row phase)
    static constexpr int RS0 = col_stride<L0, E>();       // column stride (column phase)
    static constexpr int ASZ = N0 * RS1 > N1 * RS0 ? N0 * RS1 : N1 * RS0;  // LDS per array
    static constexpr int LDS = AP * ASZ * 8;
};

template <int L0, int L1>
constexpr bool nd2_valid()
{
    using Z = Nd2Shape<L0, L1>;
    return L0 >= 1 && L1 >= 1 && L0 + L1 <= 14 && Z::TPA <= 1024 && Z::TPT1 <= 64 && Z::LDS <= 160 * 1024;
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
            my[(t + m * Z::TPT1) * Z::RS0 + r] = v[m];
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

template <int L0, int L1, int S>
hipError_t launch_nd2(const void* in, void* out, const void* rows0, const void* rows1, int64_t batch, float scale,
                      hipStream_t stream)
{
    using Z = Nd2Shape<L0, L1>;
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
        register_nd2(KernelNd2{L0, L1, Z::E, -1, Z::AP, Z::WG, &launch_nd2<L0, L1, -1>, r0, r1, Z::LDS});
        register_nd2(KernelNd2{L0, L1, Z::E, +1, Z::AP, Z::WG, &launch_nd2<L0, L1, +1>, r0, r1, Z::LDS});
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
