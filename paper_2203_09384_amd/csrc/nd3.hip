// Single-pass 3D transforms of arrays that fit one workgroup's LDS
// (N0 x N1 x N2 <= 16384 points, every axis at least 4): one HBM pass
// instead of two or three.
//
// The 3D DFT factors into a DFT along each axis in turn (its kernel is a
// product over the axes).  A workgroup holds AP whole arrays; all of an
// array's points are in registers at once (N / EPT threads, EPT points
// each), and two turns through LDS bring each axis's lines together:
//   axis 2   thread (r, t) loads points t + m TPT2 of row r (r = i0 N1 + i1)
//            straight from HBM and runs the Stockham passes in row r's own
//            LDS region (a row's threads share a wavefront);
//   turn     each result goes to LDS so that the axis-1 line (i0, i2) is
//            contiguous at stride RS1 (odd, for the banks);
//   axis 1   thread (l, t1), the line index l fastest, reads points
//            t1 + m TPT1 of line l and runs the passes in that line's place
//            (workgroup barriers: a line's threads span wavefronts);
//   turn     the results go to LDS so that the axis-0 line (i1, i2) is
//            contiguous at stride RS0;
//   axis 0   thread (c, t0), c = i1 N2 + i2 fastest, transforms line c and
//            stores X[n0][i1][i2] straight to HBM: consecutive lanes,
//            consecutive addresses.
#include "device_fft.hpp"
#include "launch.hpp"
#include "nd3.hpp"
#include "nd_maps.hpp"

#include <utility>

namespace mifft {
namespace {

template <int L0, int L1, int L2>
struct Nd3Shape {
    static constexpr ndm::Nd3Geom G = ndm::nd3_geom(L0, L1, L2);
    static constexpr int E = G.E, EPT = 1 << E;
    static constexpr int N0 = G.N0, N1 = G.N1, N2 = G.N2, N = N0 * N1 * N2;
    static constexpr int TPA = G.TPA;  // threads per array
    static constexpr int AP = G.AP;    // arrays per workgroup
    static constexpr int WG = G.WG;
    static constexpr int TPT0 = G.TPT0, TPT1 = G.TPT1, TPT2 = G.TPT2;
    static constexpr int RS2 = G.RS2;  // row stride (axis-2 phase)
    static constexpr int RS1 = G.RS1;  // axis-1 line stride
    static constexpr int RS0 = G.RS0;  // axis-0 line stride
    static constexpr int ASZ = G.ASZ;  // LDS per array
    static constexpr int LDS = G.LDS;
    static constexpr int R0 = TPT0 > 1 ? Layout2<L0, E>::rows_total() : 0;
    static constexpr int R1 = TPT1 > 1 ? Layout2<L1, E>::rows_total() : 0;
    static constexpr int R2 = TPT2 > 1 ? Layout2<L2, E>::rows_total() : 0;
};

template <int L0, int L1, int L2>
constexpr bool nd3_valid()
{
    return ndm::nd3_fits(L0, L1, L2);
}

template <int L, int E>
__device__ __forceinline__ void unit_tw(TwRegs<L, E>& tws)
{
#pragma unroll
    for (int p = 0; p < Sched<L, E>::NP; p++)
#pragma unroll
        for (int i = 0; i < (1 << E); i++)
            tws[p][i] = cf{1.f, 0.f};
}

template <int L0, int L1, int L2, int S>
__global__ __launch_bounds__((Nd3Shape<L0, L1, L2>::WG)) void k_nd3(const cf* __restrict__ in, cf* __restrict__ out,
                                                                 const cf* __restrict__ rows, int64_t batch,
                                                                 float scale)
{
    using Z = Nd3Shape<L0, L1, L2>;
    constexpr int E = Z::E, EPT = Z::EPT, N0 = Z::N0, N1 = Z::N1, N2 = Z::N2, N = Z::N;
    __shared__ cf lds[Z::AP * Z::ASZ];
    const cf* rows0 = rows;
    const cf* rows1 = rows + Z::R0;
    const cf* rows2 = rows + Z::R0 + Z::R1;
    const int tid = threadIdx.x, a = tid / Z::TPA, u = tid % Z::TPA;
    const int64_t arr = (int64_t)blockIdx.x * Z::AP + a;
    const bool live = arr < batch;
    cf* my = lds + a * Z::ASZ;
    cf v[EPT];
    // ---- axis 2 (rows r = i0 N1 + i1)
    {
        TwRegs<L2, E> tw;
        unit_tw<L2, E>(tw);
        const int r = u / Z::TPT2, t = u % Z::TPT2;
        const cf* src = in + arr * N + r * N2;
#pragma unroll
        for (int m = 0; m < EPT; m++)
            v[m] = live ? src[t + m * Z::TPT2] : cf{0.f, 0.f};
        run2<L2, E, S, 1, true>(v, t, rows2, tw, my + r * Z::RS2);
        __syncthreads();  // every row's exchanges are read
        const int i0 = r / N1, i1 = r % N1;
#pragma unroll
        for (int m = 0; m < EPT; m++)
            my[ndm::nd3_turn21(i0, i1, t + m * Z::TPT2, N2, Z::RS1)] = v[m];  // line (i0, i2), point i1
        __syncthreads();
    }
    // ---- axis 1 (lines l = i0 N2 + i2)
    {
        TwRegs<L1, E> tw;
        unit_tw<L1, E>(tw);
        constexpr int NL = N0 * N2;
        const int l = u % NL, t1 = u / NL;
        cf* line = my + l * Z::RS1;
#pragma unroll
        for (int m = 0; m < EPT; m++)
            v[m] = line[t1 + m * Z::TPT1];
        if constexpr (Z::TPT1 > 1)
            __syncthreads();  // the line is read before its exchanges overwrite it
        run2<L1, E, S, 1, false>(v, t1, rows1, tw, line);
        __syncthreads();  // every line's exchanges are read
        const int i0 = l / N2, i2 = l % N2;
#pragma unroll
        for (int m = 0; m < EPT; m++)
            my[ndm::nd3_turn10(i0, t1 + m * Z::TPT1, i2, N2, Z::RS0)] = v[m];  // line (i1, i2), point i0
        __syncthreads();
    }
    // ---- axis 0 (lines c = i1 N2 + i2), stored straight to HBM
    {
        TwRegs<L0, E> tw;
        unit_tw<L0, E>(tw);
        constexpr int NC = N1 * N2;
        const int c = u % NC, t0 = u / NC;
        cf* line = my + c * Z::RS0;
#pragma unroll
        for (int m = 0; m < EPT; m++)
            v[m] = line[t0 + m * Z::TPT0];
        if constexpr (Z::TPT0 > 1)
            __syncthreads();
        run2<L0, E, S, 1, false>(v, t0, rows0, tw, line);
        if (live) {
            cf* dst = out + arr * N + c;
#pragma unroll
            for (int m = 0; m < EPT; m++)
                dst[(t0 + m * Z::TPT0) * NC] = cscale(v[m], scale);
        }
    }
}

// Persistent form, for one array per workgroup whose axes 0 and 1 are one
// thread per line (N0 = N1 = EPT: no twiddle rows, no exchanges) and whose
// LDS leaves the CU few wavefronts to overlap loads with.  A
// workgroup walks the batch; while an array's axis-1 and axis-0 transforms
// run, the next array's rows load into registers, and the axis-2 twiddle
// rows sit in LDS (padded) for the workgroup's life, so the only global
// loads in the loop are the arrays.  The loop is rotated (the next array's
// axis 2 at the end of the body), so the wait for the prefetched rows leaves
// the stores issued before it in flight.
constexpr int ND3_ROW_PAD = 2;

template <int L0, int L1, int L2>
constexpr bool nd3_persistent()
{
    if constexpr (!nd3_valid<L0, L1, L2>()) {
        return false;
    } else {
        using Z = Nd3Shape<L0, L1, L2>;
        // only where the one-shot grid holds at most 16 wavefronts per CU
        // (LDS-bound): at 28-32 the prefetch registers cost more than the
        // overlap gains (8 x 8 x 32 188 -> 199 us, 4 x 4 x 64 185 -> 214)
        return Z::AP == 1 && Z::TPT0 == 1 && Z::TPT1 == 1 && (160 * 1024 / Z::LDS) * (Z::WG / 64) <= 16 &&
               Z::LDS + (Z::R2 > 0 ? padded_rows_total<L2, Z::E, ND3_ROW_PAD>() : 0) * 8 <= 160 * 1024;
    }
}

template <int L0, int L1, int L2, int S>
__global__ __launch_bounds__((Nd3Shape<L0, L1, L2>::WG)) void k_nd3p(const cf* __restrict__ in, cf* __restrict__ out,
                                                                  const cf* __restrict__ rows, int64_t batch,
                                                                  float scale)
{
    using Z = Nd3Shape<L0, L1, L2>;
    constexpr int E = Z::E, EPT = Z::EPT, N0 = Z::N0, N1 = Z::N1, N2 = Z::N2, N = Z::N;
    static_assert(Z::AP == 1 && Z::TPT0 == 1 && Z::TPT1 == 1, "one array per workgroup, one thread per line");
    constexpr int RP = Z::R2 > 0 ? padded_rows_total<L2, E, ND3_ROW_PAD>() : 1;
    __shared__ cf lds[Z::ASZ];
    __shared__ cf trow[RP];
    const int tid = threadIdx.x;
    int64_t g = blockIdx.x;
    if (g >= batch)
        return;
    if constexpr (Z::R2 > 0)
        copy_rows_padded<L2, E, ND3_ROW_PAD>(trow, rows, tid, Z::WG);
    TwRegs<L2, E> tw2;
    unit_tw<L2, E>(tw2);
    TwRegs<L1, E> tw1;
    unit_tw<L1, E>(tw1);
    TwRegs<L0, E> tw0;
    unit_tw<L0, E>(tw0);
    // axis 2: thread t of row r = i0 N1 + i1; axis 1: line l = i0 N2 + i2
    // (one thread each, l = tid); axis 0: line c = i1 N2 + i2 (c = tid)
    const int r = tid / Z::TPT2, t = tid % Z::TPT2;
    const int i0r = r / N1, i1r = r % N1;
    const int i0l = tid / N2, i2l = tid % N2;
    const cf* src = in + r * N2 + t;  // + g N + m TPT2: point t + m TPT2 of row r
    cf v[EPT], nx[EPT];
#pragma unroll
    for (int m = 0; m < EPT; m++)
        v[m] = src[g * N + m * Z::TPT2];
    __syncthreads();  // twiddle rows in place
    // axis 2 of x, the turn, and axis-1 line tid into v
    auto axis2_and_turn = [&](cf(&x)[EPT]) {
        run2<L2, E, S, 1, true, 0, ND3_ROW_PAD>(x, t, trow, tw2, lds + r * Z::RS2);
        __syncthreads();  // every row's exchanges are read
#pragma unroll
        for (int m = 0; m < EPT; m++)
            lds[ndm::nd3_turn21(i0r, i1r, t + m * Z::TPT2, N2, Z::RS1)] = x[m];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < EPT; m++)
            v[m] = lds[tid * Z::RS1 + m];
    };
    // axis 1 in registers, the turn, axis 0 in registers
    auto axis1_and_axis0 = [&]() {
        run2<L1, E, S, 1, false>(v, 0, rows, tw1, lds + tid * Z::RS1);
        __syncthreads();  // every axis-1 line is read
#pragma unroll
        for (int m = 0; m < EPT; m++)
            lds[ndm::nd3_turn10(i0l, m, i2l, N2, Z::RS0)] = v[m];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < EPT; m++)
            v[m] = lds[tid * Z::RS0 + m];
        run2<L0, E, S, 1, false>(v, 0, rows, tw0, lds + tid * Z::RS0);
    };
    auto store = [&]() {
        cf* dst = out + g * N + tid;
#pragma unroll
        for (int m = 0; m < EPT; m++)
            dst[m * (N1 * N2)] = cscale(v[m], scale);
    };
    const int64_t stride = gridDim.x;
    int64_t left = (batch - 1 - g) / stride;
    axis2_and_turn(v);
    while (left > 0) {
        const cf* nsrc = src + (g + stride) * N;
#pragma unroll
        for (int m = 0; m < EPT; m++)
            nx[m] = nsrc[m * Z::TPT2];
        axis1_and_axis0();
        store();
        g += stride;
        --left;
        __syncthreads();  // the axis-0 lines are read before the next array's exchanges and turn
        axis2_and_turn(nx);
    }
    axis1_and_axis0();
    store();
}

template <int L0, int L1, int L2, int S>
int nd3_slots()
{
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 0;
    if (cached[dev] == 0) {
        int cus = 0, per = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_nd3p<L0, L1, L2, S>, Nd3Shape<L0, L1, L2>::WG, 0) !=
                hipSuccess)
            return 0;
        cached[dev] = cus * per;
    }
    return cached[dev];
}

template <int L0, int L1, int L2, int S>
hipError_t launch_nd3(const void* in, void* out, const void* rows, int64_t batch, float scale, hipStream_t stream)
{
    using Z = Nd3Shape<L0, L1, L2>;
    if constexpr (nd3_persistent<L0, L1, L2>()) {
        const int slots = nd3_slots<L0, L1, L2, S>();
        if (slots > 0) {
            const int64_t grid = batch > slots ? slots : batch;
            return launch_kernel((k_nd3p<L0, L1, L2, S>), dim3((unsigned)grid), dim3(Z::WG), 0, stream,
                                 static_cast<const cf*>(in), static_cast<cf*>(out), static_cast<const cf*>(rows),
                                 batch, scale);
        }
    }
    const int64_t grid = (batch + Z::AP - 1) / Z::AP;
    return launch_kernel((k_nd3<L0, L1, L2, S>), dim3((unsigned)grid), dim3(Z::WG), 0, stream,
                         static_cast<const cf*>(in), static_cast<cf*>(out), static_cast<const cf*>(rows), batch, scale);
}

template <int L0, int L1, int L2, int S>
constexpr auto nd3_slots_fn()
{
    if constexpr (nd3_persistent<L0, L1, L2>())
        return &nd3_slots<L0, L1, L2, S>;
    else
        return static_cast<int (*)()>(nullptr);
}

template <int L0, int L1, int L2>
void add_nd3()
{
    if constexpr (nd3_valid<L0, L1, L2>()) {
        using Z = Nd3Shape<L0, L1, L2>;
        constexpr int lds = Z::LDS + (nd3_persistent<L0, L1, L2>() && Z::R2 > 0
                                          ? padded_rows_total<L2, Z::E, ND3_ROW_PAD>() * 8
                                          : 0);
        register_nd3(KernelNd3{{L0, L1, L2}, Z::E, -1, Z::AP, Z::WG, &launch_nd3<L0, L1, L2, -1>, {Z::R0, Z::R1, Z::R2},
                               lds, nd3_slots_fn<L0, L1, L2, -1>()});
        register_nd3(KernelNd3{{L0, L1, L2}, Z::E, +1, Z::AP, Z::WG, &launch_nd3<L0, L1, L2, +1>, {Z::R0, Z::R1, Z::R2},
                               lds, nd3_slots_fn<L0, L1, L2, +1>()});
    }
}

// every (L0, L1, L2) with each in [2, 10] and L0 + L1 + L2 <= 14
template <int L0, int L1, int... L2s>
void add_l2(std::integer_sequence<int, L2s...>)
{
    (add_nd3<L0, L1, L2s + 2>(), ...);
}

template <int L0, int... L1s>
void add_l1(std::integer_sequence<int, L1s...>)
{
    (add_l2<L0, L1s + 2>(std::make_integer_sequence<int, 9>{}), ...);
}

template <int... L0s>
void add_l0(std::integer_sequence<int, L0s...>)
{
    (add_l1<L0s + 2>(std::make_integer_sequence<int, 9>{}), ...);
}

struct Nd3Registrar {
    Nd3Registrar() { add_l0(std::make_integer_sequence<int, 9>{}); }
};
Nd3Registrar nd3_registrar;

}  // namespace
}  // namespace mifft
