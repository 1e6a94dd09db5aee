// Lengths 2^12 .. 2^20 (FP32): four-step Cooley-Tukey split N = N1 * N2.
//
// With n = n1 N2 + n2 and k = k1 + N1 k2 the DFT of Eq. (dft) factors as
//   X[k1 + N1 k2] = sum_n2 w_N2^{n2 k2} ( w_N^{n2 k1} sum_n1 x[n1 N2 + n2] w_N1^{n1 k1} )
// i.e. the radix-N1 / radix-N2 Cooley-Tukey split of Eq. (radix2) taken
// once with large radices.  Two kernels:
//   pass 1  column DFTs of length N1 (stride N2) times w_N^{n2 k1}, stored
//           to Y[k1 + N1 n2] of `out` (so pass 2's tile is read and written
//           in place);
//   pass 2  row DFTs of length N2 over n2, in place in `out`, output
//           X[k1 + N1 k2] (times the plan's scale).
// Each workgroup owns a tile of 16 transforms (16 columns, or 16 rows k1)
// so that every global load and store is a run of 16 complex values (one
// 128-byte line), and transforms them with the same Stockham passes as the
// batched kernels.  Long inner transforms are read straight into registers
// (the tile's transform index is the fastest lane index); short ones are
// staged through LDS so that their exchanges stay inside one wavefront.
// w_N^j is built from a two-level FP32 table (w_N^{1024 a} and w_N^{b},
// both from FP64 sincospi); the column pass reads it as three levels in LDS.
#include "device_fft.hpp"
#include "launch.hpp"
#include "fourstep.hpp"
#include "tile_fft.hpp"

namespace mifft {
namespace {

constexpr int TILE = 16;

template <int S>
__device__ __forceinline__ cf big_twiddle(const cf* __restrict__ lo, const cf* __restrict__ hi, unsigned j)
{
    cf w = cmul(hi[j >> 10], lo[j & 1023u]);
    if constexpr (S > 0)
        w.y = -w.y;
    return w;
}

// The w_N^{n2 k1} lookups are gathers (every lane its own entry); from the
// cached two-level table they cost about a tenth of the four-step's time.
// Each workgroup copies a three-level table into LDS instead (w_N^{1024 a},
// w_N^{32 b}, w_N^{c} for j = 1024 a + 32 b + c: 64 + N / 1024 entries, at
// most 8.5 KiB, taken from the two-level table), at one more complex product
// per point and without losing a workgroup per CU.  MI355X, 2^26 elements:
// 2^15 468 -> 428 us, 2^16 483 -> 440, 2^17 519 -> 478, 2^18 525 -> 485,
// 2^19 552 -> 508, 2^20 567 -> 542.  (The two levels whole in LDS, 10 KiB at
// 2^18, cost a workgroup per CU at 256-point columns.)
constexpr bool tw3_in_lds(int L) { return L >= 15; }

// Columns per pass-1 tile: 16 (whole 128-byte lines), or 8 for 1024-point
// columns so that two workgroups fit one CU's LDS (MI355X, 2^26 elements:
// 2^20 616 -> 578 us, 2^19 583 -> 547 us).
constexpr int col_tile(int L1) { return L1 >= 10 ? 8 : 16; }
// Columns of 128+ points load straight into registers (MI355X: 2^15
// 485 -> 468 us, 2^16 494 -> 479 us against staging 128- and 256-point
// columns through LDS); the row pass keeps the axis-pass threshold.
constexpr bool col_direct(int L1) { return L1 >= 7; }

// Pass 1: tile = columns n2 in [T nb, T nb + T) of transform b (T =
// col_tile).  Long columns (col_direct) are read straight into registers
// (the column index is the fastest lane index: rows of T values per
// wavefront access); short ones are staged through LDS so their exchanges
// stay inside one wavefront.  Either way the outputs go out through LDS:
// the tile's outputs Y[k1 + N1 n2] form one contiguous block.
template <int L1, int L2, int S>
__global__ __launch_bounds__(col_tile(L1)*((1 << L1) >> inner_e(L1))) void k_fourstep1(
    const cf* __restrict__ in, cf* __restrict__ out, const cf* __restrict__ rows, const cf* __restrict__ tlo,
    const cf* __restrict__ thi, int64_t ntiles)
{
    constexpr int T = col_tile(L1), LT = T == 16 ? 4 : 3;
    constexpr int E = inner_e(L1), N1 = 1 << L1, N2 = 1 << L2;
    constexpr int EPT = 1 << E, TPT = N1 / EPT, WG = T * TPT, ST = stage_stride<L1, E>();
    constexpr bool DIRECT = col_direct(L1);
    static_assert(T == 16 || DIRECT, "8-column tiles load directly");
    // the three-level table in LDS (tw3_in_lds): twl[c], twl[32 + b],
    // twl[64 + a]
    constexpr bool TW3 = tw3_in_lds(L1 + L2);
    constexpr int NHI = (1 << (L1 + L2)) >> 10;
    constexpr int NTW = TW3 ? 64 + NHI : 1;
    __shared__ cf lds[T * ST];
    __shared__ cf twl[NTW];
    const int tid = threadIdx.x;
    int64_t tile = blockIdx.x;
    if constexpr (T < 16) {
        // tiles 2i and 2i+1 share 128-byte lines: same XCD (blocks b, b + 8)
        const int64_t g = blockIdx.x;
        tile = idx::xcd_group_tile(g, 2);
    }
    if (tile >= ntiles)
        return;
    const int nb = (int)(tile % (N2 / T));
    // thread (tb, t): transform tb of the tile, thread t of that transform
    const int tb = DIRECT ? (tid & (T - 1)) : tid / TPT;
    const int t = DIRECT ? (tid >> LT) : tid % TPT;
    cf* my = lds + tb * ST;
    cf v[EPT];
    if constexpr (DIRECT) {
#pragma unroll
        for (int m = 0; m < EPT; m++)
            v[m] = ld_c(in + idx::fourstep_col_in(tile, tb, t + m * TPT, L1, L2, T));
    } else {
        // stage: 16 consecutive columns per row n1 (one 128-byte line)
#pragma unroll
        for (int i = 0; i < T * N1 / WG; i++) {
            const int w = tid + i * WG;
            const int c = w & (T - 1), n1 = w >> LT;
            lds[c * ST + n1] = ld_c(in + idx::fourstep_col_in(tile, c, n1, L1, L2, T));
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < EPT; m++)
            v[m] = my[t + m * TPT];
    }
    if constexpr (TW3) {
        // twl: w_N^c (c < 32), w_N^{32 b} (b < 32), then w_N^{1024 a}
        for (int i = tid; i < NTW; i += WG)
            twl[i] = i < 32 ? tlo[i] : i < 64 ? tlo[32 * (i - 32)] : thi[i - 64];
        __syncthreads();
    }
    TwRegs<L1, E> tws;
    unit_rows<L1, E>(tws);
    constexpr bool WAVE = DIRECT ? TPT * T <= 64 : TPT <= 64;
    run2<L1, E, S, 1, WAVE>(v, t, rows, tws, my);
    const unsigned n2 = nb * T + tb;
#pragma unroll
    for (int m = 0; m < EPT; m++) {
        const unsigned k1 = t + m * TPT;
        const unsigned j = n2 * k1;
        cf w;
        if constexpr (TW3) {
            w = cmul(cmul(twl[64 + (j >> 10)], twl[32 + ((j >> 5) & 31u)]), twl[j & 31u]);
            if constexpr (S > 0)
                w.y = -w.y;
        } else {
            w = big_twiddle<S>(tlo, thi, j);
        }
        v[m] = cmul(v[m], w);
    }
    if constexpr (DIRECT)
        __syncthreads();  // every transform's last exchange is read
    else
        lds_sync<true>();  // this wavefront's last exchange is read
#pragma unroll
    for (int m = 0; m < EPT; m++)
        my[t + m * TPT] = v[m];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < T * N1 / WG; i++) {
        const int w = tid + i * WG;
        const int c = w / N1, k1 = w % N1;
        st_c(out + idx::fourstep_col_out(tile, c, k1, L1, L2, T), lds[c * ST + k1]);
    }
}

// Pass 2 (in place): tile = rows k1 in [16 kb, 16 kb + 16) of transform b,
// elements Y[k1 + N1 n2] (stride N1 along n2); outputs X[k1 + N1 k2] at the
// same addresses: the axis pass of a multidimensional transform with
// stride N1 over batch * N1 transforms.
template <int L1, int L2, int S>
__global__ __launch_bounds__(axis_wg<L2>()) void k_fourstep2(cf* __restrict__ io, const cf* __restrict__ rows,
                                                            int64_t count, float scale)
{
    static_assert(axis_tile(L2) == TILE, "row tiles of 16");
    __shared__ cf lds[TILE * stage_stride<L2, axis_e(L2)>()];
    const int64_t q0 = (int64_t)blockIdx.x * TILE;
    if constexpr (axis_direct(L2))
        axis_tile_direct<L2, S>(io, rows, lds, q0, count, L1, scale);
    else
        axis_tile_staged<L2, S>(io, rows, lds, q0, count, L1, scale);
}

template <int L1, int L2, int S>
hipError_t launch_fourstep(const void* in, void* out, const void* rows1, const void* rows2, const void* tlo,
                           const void* thi, int64_t batch, float scale, hipStream_t stream)
{
    constexpr int T1 = col_tile(L1);
    constexpr int WG1 = T1 * ((1 << L1) >> inner_e(L1));
    constexpr int WG2 = TILE * ((1 << L2) >> inner_e(L2));
    const int64_t t1 = batch * ((1 << L2) / T1), g2 = batch * ((1 << L1) / TILE);
    const int64_t g1 = T1 < 16 ? (t1 + 15) & ~int64_t(15) : t1;  // whole chunks for the XCD pairing
    const hipError_t e = launch_kernel((k_fourstep1<L1, L2, S>), dim3((unsigned)g1), dim3(WG1), 0, stream,
                                       static_cast<const cf*>(in), static_cast<cf*>(out),
                                       static_cast<const cf*>(rows1), static_cast<const cf*>(tlo),
                                       static_cast<const cf*>(thi), t1);
    if (e != hipSuccess)
        return e;
    // pass 2 is the axis pass of stride N1 over batch N1 transforms: the
    // persistent form where it applies (1024-point rows)
    hipError_t e2;
    if (launch_axis_persistent<L2, S>(out, rows2, batch << L1, L1, scale, stream, &e2))
        return e2;
    return launch_kernel((k_fourstep2<L1, L2, S>), dim3((unsigned)g2), dim3(WG2), 0, stream, static_cast<cf*>(out),
                       static_cast<const cf*>(rows2), batch << L1, scale);
}

template <int L>
void add_len()
{
    constexpr int L1 = (L + 1) / 2, L2 = L / 2;
    const FourStep fs{L, L1, L2, inner_e(L1), inner_e(L2), Layout2<L1, inner_e(L1)>::rows_total(),
                      Layout2<L2, inner_e(L2)>::rows_total(), &launch_fourstep<L1, L2, -1>,
                      &launch_fourstep<L1, L2, +1>,
                      (int)((col_tile(L1) * stage_stride<L1, inner_e(L1)>() +
                             (tw3_in_lds(L) ? 64 + (1 << (L - 10)) : 0)) *
                            sizeof(cf)),
                      (int)(TILE * stage_stride<L2, inner_e(L2)>() * sizeof(cf)), col_tile(L1)};
    register_fourstep(fs);
}

struct FourStepRegistrar {
    FourStepRegistrar()
    {
        add_len<12>();
        add_len<13>();
        add_len<14>();
        add_len<15>();
        add_len<16>();
        add_len<17>();
        add_len<18>();
        add_len<19>();
        add_len<20>();
    }
};
FourStepRegistrar fourstep_registrar;

}  // namespace

// Two-level twiddles of length N = 2^L: lo[b] = w_N^b (b < 1024),
// hi[a] = w_N^{1024 a} (a < N / 1024), w_N = exp(-2 pi i / N), FP64 sincospi
// rounded once to FP32.
__global__ void k_twiddle_big(float2* __restrict__ lo, float2* __restrict__ hi, int L)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int nhi = 1 << (L - 10);
    if (i >= 1024 + nhi)
        return;
    const int64_t j = i < 1024 ? i : (int64_t)(i - 1024) << 10;
    double s, c;
    sincospi(2.0 * (double)j / (double)(int64_t(1) << L), &s, &c);
    const float2 w = float2{(float)c, (float)(-s)};
    if (i < 1024)
        lo[i] = w;
    else
        hi[i - 1024] = w;
}

hipError_t launch_twiddle_big(void* lo, void* hi, int L, hipStream_t stream)
{
    const int total = 1024 + (1 << (L - 10));
    return launch_kernel(k_twiddle_big, dim3((total + 255) / 256), dim3(256), 0, stream, static_cast<float2*>(lo),
                       static_cast<float2*>(hi), L);
}

}  // namespace mifft
