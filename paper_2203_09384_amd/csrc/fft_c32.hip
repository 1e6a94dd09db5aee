// FP32 interleaved complex batched Stockham FFT kernels, one translation
// unit per transform length: this file is compiled once per log2(N) with
// -DMIFFT_LOG2N=<1..11> and registers every (EPT, workgroup size, sign)
// variant it instantiates with the host-side kernel registry.
//
// Workgroup layout: TPT = N/EPT threads per transform, TPB = WG/TPT
// transforms per workgroup, one transform per TPT consecutive threads.
// Thread t of a transform loads x[t + m TPT] for m < EPT (each wave load
// instruction covers whole 64-lane runs of consecutive complex values),
// runs every pass in registers with LDS exchanges in between, and stores
// X[t + m TPT] (natural order), multiplied by the plan's scale.
#include "device_fft.hpp"
#include "launch.hpp"
#include "registry.hpp"

#ifndef MIFFT_LOG2N
#error "compile with -DMIFFT_LOG2N=<1..14>"
#endif

namespace mifft {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ v4f ld_data4(const gv4* p)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

template <bool NT>
__device__ __forceinline__ void st_data4(gv4* p, v4f v)
{
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <int LOG2N, int LOG2EPT, int WG, int S>
__global__ __launch_bounds__(WG) void k_fft_c32(const cf* __restrict__ in, cf* __restrict__ out,
                                                const cf* __restrict__ tw, int64_t batch, float scale)
{
    using SC = Sched<LOG2N, LOG2EPT>;
    constexpr int N = SC::N, EPT = SC::EPT, TPT = SC::TPT, TPB = WG / TPT;
    constexpr bool NT = stream_nt<N, TPT>();
    const int tid = threadIdx.x;
    const int tb = tid / TPT, t = tid % TPT;
    const int64_t b = (int64_t)blockIdx.x * TPB + tb;
    const bool live = b < batch;
    const cf* __restrict__ src = in + b * N;
    cf* __restrict__ dst = out + b * N;
    cf v[EPT];

    if constexpr (TPT == 1) {
        // One thread owns a whole (short) transform: 16-byte vector loads of
        // consecutive elements, a single in-register DFT, no LDS.
        static_assert(SC::NP == 1, "single pass expected");
        if (live) {
            const gv4* s4 = reinterpret_cast<const gv4*>(src);
#pragma unroll
            for (int m = 0; m < EPT / 2; m++) {
                const v4f q = ld_data4<NT>(s4 + m);
                v[2 * m] = cf{q.x, q.y};
                v[2 * m + 1] = cf{q.z, q.w};
            }
        } else {
#pragma unroll
            for (int m = 0; m < EPT; m++)
                v[m] = cf{0.f, 0.f};
        }
        pass_compute<LOG2N, LOG2EPT, S, 0>(v, 0, tw);
        if (live) {
            gv4* d4 = reinterpret_cast<gv4*>(dst);
#pragma unroll
            for (int m = 0; m < EPT / 2; m++) {
                v4f q;
                q.x = v[2 * m].x * scale;
                q.y = v[2 * m].y * scale;
                q.z = v[2 * m + 1].x * scale;
                q.w = v[2 * m + 1].y * scale;
                st_data4<NT>(d4 + m, q);
            }
        }
    } else {
        __shared__ float lre[TPB * N];
        __shared__ float lim[TPB * N];
#pragma unroll
        for (int m = 0; m < EPT; m++)
            v[m] = live ? ld_data<NT>(reinterpret_cast<const char*>(src + t + m * TPT)) : cf{0.f, 0.f};
        run_passes<LOG2N, LOG2EPT, S>(v, t, tw, lre + tb * N, lim + tb * N);
        if (live) {
#pragma unroll
            for (int m = 0; m < EPT; m++)
                st_data<NT>(reinterpret_cast<char*>(dst + t + m * TPT), cscale(v[m], scale));
        }
    }
}

// ---------------------------------------------------------------- v2
// Persistent, pipelined variant.  Each workgroup walks the transform groups
// g = blockIdx.x, blockIdx.x + gridDim.x, ...; TPB transforms per group.
//   TW = 0: the thread's twiddle rows for every pass are loaded once and kept
//           in VGPRs (they depend on the thread index only);
//   TW = 1: they are re-read (from L1/L2) for every group.
//   PF = 1: the next group's input is loaded into a second register set
//           while the current group is transformed and stored.
// Global addresses are a uniform (SGPR) group base plus a 32-bit per-thread
// byte offset; LDS addresses are one per-thread base plus immediates.

template <int L, int E, int WG, int S, int TW, int PF, bool WAVE>
__global__ __launch_bounds__(WG) void k_fft_c32_v2(const cf* __restrict__ in, cf* __restrict__ out,
                                                   const cf* __restrict__ rows, int64_t batch, float scale)
{
    using SC = Sched<L, E>;
    constexpr int N = SC::N, EPT = SC::EPT, TPT = SC::TPT, TPB = WG / TPT, NP = SC::NP;
    constexpr int REG = Layout2<L, E>::region();
    static_assert(TPT >= 2, "v2 needs an LDS exchange");
    static_assert(!WAVE || TPT <= 64, "wave-local exchanges need a transform inside one wavefront");
    __shared__ cf lds[TPB * REG];
    const int tid = threadIdx.x, tb = tid / TPT, t = tid % TPT;
    cf* my = lds + tb * REG;
    const unsigned toff8 = (unsigned)(tb * N + t) * 8u;
    const int64_t ngroups = (batch + TPB - 1) / TPB;
    int64_t g = blockIdx.x;
    if (g >= ngroups)
        return;
    cf tws[NP][EPT];
#pragma unroll
    for (int p = 0; p < NP; p++)
#pragma unroll
        for (int r = 0; r < EPT; r++)
            tws[p][r] = cf{1.f, 0.f};
    if constexpr (TW == 0)
        load_all_rows<L, E, S>(tws, rows, t);
    cf a[EPT], b[EPT];
    load_group<L, E, TPB>(a, in, g, batch, tb, toff8);
    if constexpr (!PF) {
        // one group per workgroup (the grid covers every group)
        run2<L, E, S, TW, WAVE>(a, t, rows, tws, my);
        store_group<L, E, TPB>(a, out, g, batch, tb, toff8, scale);
        return;
    }
    // Groups g, g + stride, ... ; `left` more after the current one.  The
    // loop body issues the next group's loads unconditionally (two groups
    // per trip, one per register set), a slice before each pass, and the
    // last one or two groups run after it.  A prefetch under a condition
    // would let the path without it meet the path with it before the
    // current group is used, and the wait placed there would then cover
    // most of the prefetched loads.
    //
    // The loop is rotated so that its head is the b body: both edges into it
    // come from an a body that has just issued b's loads and then a's
    // stores, so the wait for b leaves those stores in flight.  (With the a
    // body at the head, the edge from before the loop, where no stores are
    // outstanding, would make that wait cover the stores on every trip.)
    const int64_t stride = gridDim.x;
    int64_t left = (ngroups - 1 - g) / stride;
    if (left >= 2) {
        run2_prefetch<L, E, S, TW, WAVE, TPB>(a, t, rows, tws, my, b, in, g + stride, batch, tb, toff8);
        store_group<L, E, TPB>(a, out, g, batch, tb, toff8, scale);
        g += stride;
        lds_sync<WAVE>();  // LDS is reused by the next group
        while (true) {
            run2_prefetch<L, E, S, TW, WAVE, TPB>(b, t, rows, tws, my, a, in, g + stride, batch, tb, toff8);
            store_group<L, E, TPB>(b, out, g, batch, tb, toff8, scale);
            g += stride;
            lds_sync<WAVE>();
            left -= 2;
            if (left < 2)
                break;
            run2_prefetch<L, E, S, TW, WAVE, TPB>(a, t, rows, tws, my, b, in, g + stride, batch, tb, toff8);
            store_group<L, E, TPB>(a, out, g, batch, tb, toff8, scale);
            g += stride;
            lds_sync<WAVE>();
        }
    }
    if (left == 1) {
        run2_prefetch<L, E, S, TW, WAVE, TPB>(a, t, rows, tws, my, b, in, g + stride, batch, tb, toff8);
        store_group<L, E, TPB>(a, out, g, batch, tb, toff8, scale);
        g += stride;
        lds_sync<WAVE>();
        run2<L, E, S, TW, WAVE>(b, t, rows, tws, my);
        store_group<L, E, TPB>(b, out, g, batch, tb, toff8, scale);
    } else {
        run2<L, E, S, TW, WAVE>(a, t, rows, tws, my);
        store_group<L, E, TPB>(a, out, g, batch, tb, toff8, scale);
    }
}

// ---------------------------------------------------------------- staged
// Short lengths (N <= 16), one transform per thread, with the workgroup's
// block of WG transforms moved between HBM and LDS in 16-byte vectors at
// consecutive lane addresses: each wave instruction covers 1 KiB of
// contiguous input or output.  In LDS each transform is a row of N/2
// vectors, padded by one vector when N >= 4 so that the per-thread row
// accesses hit distinct banks.  A thread reads its row, transforms it in
// registers, writes its row back (no other thread touches it), and the
// block leaves LDS the way it came in.
template <int L, int WG, int S>
__global__ __launch_bounds__(WG) void k_fft_c32_st(const cf* __restrict__ in, cf* __restrict__ out,
                                                   const cf* __restrict__ tw, int64_t batch, float scale)
{
    constexpr int N = 1 << L, H = N / 2, ROW = H + (H >= 2 ? 1 : 0);
    static_assert(L >= 1 && L <= 4, "one transform per thread: N = 2..16");
    __shared__ v4f lds[WG * ROW];
    const int tid = threadIdx.x;
    const int64_t first = (int64_t)blockIdx.x * WG;
    const int64_t count = batch - first < WG ? batch - first : WG;  // transforms of this workgroup
    const int nv = (int)count * H;                                   // its 16-byte vectors
    const gv4* src = reinterpret_cast<const gv4*>(in + first * N);
    gv4* dst = reinterpret_cast<gv4*>(out + first * N);
    v4f q[H];
    if (count == WG) {  // every load of the block issued before any is used
#pragma unroll
        for (int k = 0; k < H; k++)
            q[k] = __builtin_nontemporal_load(src + tid + WG * k);
    } else {
#pragma unroll
        for (int k = 0; k < H; k++)
            q[k] = tid + WG * k < nv ? __builtin_nontemporal_load(src + tid + WG * k) : v4f{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int k = 0; k < H; k++) {
        const int i = tid + WG * k;
        lds[(i / H) * ROW + i % H] = q[k];
    }
    __syncthreads();
    cf v[N];
#pragma unroll
    for (int j = 0; j < H; j++) {
        const v4f q = lds[tid * ROW + j];
        v[2 * j] = cf{q.x, q.y};
        v[2 * j + 1] = cf{q.z, q.w};
    }
    pass_compute<L, L, S, 0>(v, 0, tw);
#pragma unroll
    for (int j = 0; j < H; j++)
        lds[tid * ROW + j] = v4f{v[2 * j].x * scale, v[2 * j].y * scale, v[2 * j + 1].x * scale,
                                 v[2 * j + 1].y * scale};
    __syncthreads();
#pragma unroll
    for (int k = 0; k < H; k++) {
        const int i = tid + WG * k;
        q[k] = lds[(i / H) * ROW + i % H];
    }
    if (count == WG) {
#pragma unroll
        for (int k = 0; k < H; k++)
            __builtin_nontemporal_store(q[k], dst + tid + WG * k);
    } else {
#pragma unroll
        for (int k = 0; k < H; k++)
            if (tid + WG * k < nv)
                __builtin_nontemporal_store(q[k], dst + tid + WG * k);
    }
}

// The same staging for short lengths shared by TPT = N/EPT threads (at most
// one wavefront): after the block is in LDS, thread t of a transform reads
// its elements t + m TPT from the row, runs the passes with wavefront-local
// exchanges in a separate region, and writes them back to the row.
template <int L, int E, int WG, int S>
__global__ __launch_bounds__(WG) void k_fft_c32_st2(const cf* __restrict__ in, cf* __restrict__ out,
                                                    const cf* __restrict__ rows, int64_t batch, float scale)
{
    using SC = Sched<L, E>;
    constexpr int N = SC::N, EPT = SC::EPT, TPT = SC::TPT, TPB = WG / TPT, NP = SC::NP;
    constexpr int H = N / 2, ROW = H + 1, RC = 2 * ROW;  // row length in vectors / complex values
    constexpr int REG = Layout2<L, E>::region();
    static_assert(TPT >= 2 && TPT <= 64, "transforms of 2..64 threads");
    __shared__ v4f blk[TPB * ROW];
    __shared__ cf xch[TPB * REG];
    const int tid = threadIdx.x, tb = tid / TPT, t = tid % TPT;
    const int64_t first = (int64_t)blockIdx.x * TPB;
    const int64_t count = batch - first < TPB ? batch - first : TPB;
    const int nv = (int)count * H;
    const gv4* src = reinterpret_cast<const gv4*>(in + first * N);
    gv4* dst = reinterpret_cast<gv4*>(out + first * N);
    constexpr int K = TPB * H / WG;  // vectors per thread = EPT / 2
    cf tws[NP][EPT];
#pragma unroll
    for (int p = 0; p < NP; p++)
#pragma unroll
        for (int r = 0; r < EPT; r++)
            tws[p][r] = cf{1.f, 0.f};
    load_all_rows<L, E, S>(tws, rows, t);
    v4f q[K];
    if (count == TPB) {
#pragma unroll
        for (int k = 0; k < K; k++)
            q[k] = __builtin_nontemporal_load(src + tid + WG * k);
    } else {
#pragma unroll
        for (int k = 0; k < K; k++)
            q[k] = tid + WG * k < nv ? __builtin_nontemporal_load(src + tid + WG * k) : v4f{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int k = 0; k < K; k++) {
        const int i = tid + WG * k;
        blk[(i / H) * ROW + i % H] = q[k];
    }
    __syncthreads();
    cf* row = reinterpret_cast<cf*>(blk) + tb * RC;
    cf v[EPT];
#pragma unroll
    for (int m = 0; m < EPT; m++)
        v[m] = row[t + m * TPT];
    run2<L, E, S, 0, true>(v, t, rows, tws, xch + tb * REG);
#pragma unroll
    for (int m = 0; m < EPT; m++)
        row[t + m * TPT] = cscale(v[m], scale);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; k++) {
        const int i = tid + WG * k;
        q[k] = blk[(i / H) * ROW + i % H];
    }
    if (count == TPB) {
#pragma unroll
        for (int k = 0; k < K; k++)
            __builtin_nontemporal_store(q[k], dst + tid + WG * k);
    } else {
#pragma unroll
        for (int k = 0; k < K; k++)
            if (tid + WG * k < nv)
                __builtin_nontemporal_store(q[k], dst + tid + WG * k);
    }
}

template <int L, int E, int WG, int S>
hipError_t launch_c32_st2(const void* in, void* out, const void*, const void* rows, int64_t batch, float scale,
                          int64_t, hipStream_t stream)
{
    constexpr int TPB = WG / Sched<L, E>::TPT;
    const int64_t grid = (batch + TPB - 1) / TPB;
    return launch_kernel((k_fft_c32_st2<L, E, WG, S>), dim3((unsigned)grid), dim3(WG), 0, stream,
                       static_cast<const cf*>(in), static_cast<cf*>(out), static_cast<const cf*>(rows), batch,
                       scale);
}

template <int L, int WG, int S>
hipError_t launch_c32_st(const void* in, void* out, const void* tw, const void*, int64_t batch, float scale,
                         int64_t, hipStream_t stream)
{
    const int64_t grid = (batch + WG - 1) / WG;
    return launch_kernel((k_fft_c32_st<L, WG, S>), dim3((unsigned)grid), dim3(WG), 0, stream,
                       static_cast<const cf*>(in), static_cast<cf*>(out), static_cast<const cf*>(tw), batch, scale);
}

template <int LOG2N, int LOG2EPT, int WG, int S>
hipError_t launch_c32(const void* in, void* out, const void* tw, const void*, int64_t batch, float scale,
                      int64_t, hipStream_t stream)
{
    constexpr int TPB = WG / Sched<LOG2N, LOG2EPT>::TPT;
    const int64_t grid = (batch + TPB - 1) / TPB;
    return launch_kernel((k_fft_c32<LOG2N, LOG2EPT, WG, S>), dim3((unsigned)grid), dim3(WG), 0, stream,
                       static_cast<const cf*>(in), static_cast<cf*>(out), static_cast<const cf*>(tw), batch,
                       scale);
}

// grid_limit > 0 caps the number of (persistent) workgroups.
template <int L, int E, int WG, int S, int TW, int PF, bool WAVE>
hipError_t launch_c32_v2(const void* in, void* out, const void*, const void* rows, int64_t batch, float scale,
                         int64_t grid_limit, hipStream_t stream)
{
    constexpr int TPB = WG / Sched<L, E>::TPT;
    int64_t grid = (batch + TPB - 1) / TPB;
    if (grid_limit > 0 && grid > grid_limit)
        grid = grid_limit;
    return launch_kernel((k_fft_c32_v2<L, E, WG, S, TW, PF, WAVE>), dim3((unsigned)grid), dim3(WG), 0, stream,
                       static_cast<const cf*>(in), static_cast<cf*>(out), static_cast<const cf*>(rows), batch,
                       scale);
}

template <int L, int E, int WG, int S, int TW, int PF, bool WAVE>
int occupancy_v2()
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_fft_c32_v2<L, E, WG, S, TW, PF, WAVE>, WG, 0) !=
        hipSuccess)
        return 0;
    return blocks;
}

// Variant menu, v1: EPT in {2,4,8,16} (not above N; at least 4 once
// N >= 64), WG in {64,128,256,512}, TPT <= WG, LDS per workgroup <= 64 KiB;
// a thread owns a whole transform (TPT = 1) only for N <= 16.
template <int LOG2N, int LOG2EPT, int WG>
constexpr bool valid_cfg()
{
    if constexpr (LOG2EPT > LOG2N || LOG2N > 11) {
        return false;
    } else {
        constexpr int TPT = (1 << LOG2N) >> LOG2EPT;
        if (LOG2N >= 6 && LOG2EPT < 2) return false;
        if (TPT > WG) return false;
        if (TPT == 1 && LOG2N > 4) return false;
        if (TPT > 1 && (WG << LOG2EPT) * 8 > 65536) return false;
        return true;
    }
}

// v2: EPT in {4, 8, 16}, at least two threads per transform, WG <= 256
// and LDS <= 64 KiB; lengths above 2048 (up to 2^14): EPT 8 or 16, one
// transform per workgroup of up to 1024 threads and up to 160 KiB of LDS.
template <int L, int E, int WG>
constexpr bool valid_v2()
{
    if constexpr (E < 2 || E >= L) {
        return false;
    } else if constexpr (L > 11) {
        constexpr int TPT = (1 << L) >> E;
        return E >= 3 && TPT == WG && WG <= 1024 && Layout2<L, E>::region() * 8 <= 160 * 1024;
    } else if constexpr (WG > 256) {
        return false;
    } else {
        constexpr int TPT = (1 << L) >> E;
        if constexpr (TPT > WG)
            return false;
        else
            return (WG / TPT) * Layout2<L, E>::region() * 8 <= 65536;
    }
}

template <int LOG2N, int LOG2EPT, int WG, int S>
void add_one()
{
    if constexpr (valid_cfg<LOG2N, LOG2EPT, WG>())
        register_c32(KernelC32{LOG2N, LOG2EPT, WG, S, 0, &launch_c32<LOG2N, LOG2EPT, WG, S>, nullptr, 0,
                               ((1 << LOG2N) >> LOG2EPT) > 1 ? WG * (1 << LOG2EPT) * 8 : 0});
}

template <int L, int E, int WG, int S, int TW, int PF>
void add_v2()
{
    if constexpr (valid_v2<L, E, WG>()) {
        register_c32(KernelC32{L, E, WG, S, 1 + TW + 2 * PF, &launch_c32_v2<L, E, WG, S, TW, PF, false>,
                               &occupancy_v2<L, E, WG, S, TW, PF, false>, Layout2<L, E>::rows_total(),
                               (WG / ((1 << L) >> E)) * Layout2<L, E>::region() * 8});
        if constexpr (((1 << L) >> E) <= 64)
            register_c32(KernelC32{L, E, WG, S, 5 + TW + 2 * PF, &launch_c32_v2<L, E, WG, S, TW, PF, true>,
                                   &occupancy_v2<L, E, WG, S, TW, PF, true>, Layout2<L, E>::rows_total(),
                                   (WG / ((1 << L) >> E)) * Layout2<L, E>::region() * 8});
    }
}

// kind 11: the staged one-transform-per-thread kernel, N = 2..16, EPT = N,
// 64..256 threads
template <int LOG2N, int LOG2EPT, int WG, int S>
void add_st()
{
    if constexpr (LOG2N >= 1 && LOG2N <= 4 && LOG2EPT == LOG2N && WG <= 256)
        register_c32(KernelC32{LOG2N, LOG2EPT, WG, S, 11, &launch_c32_st<LOG2N, WG, S>, nullptr, 0,
                               WG * ((1 << LOG2N) / 2 + ((1 << LOG2N) >= 4 ? 1 : 0)) * 16});
}

// kind 12: staged, several threads per transform (N = 32 .. 1024), 64..256 threads
template <int L, int E, int WG, int S>
void add_st2()
{
    if constexpr (L >= 5 && L <= 10 && E >= 2 && E < L && WG <= 256) {
        constexpr int TPT = (1 << L) >> E;
        if constexpr (TPT >= 2 && TPT <= 64 && TPT <= WG)
            register_c32(KernelC32{L, E, WG, S, 12, &launch_c32_st2<L, E, WG, S>, nullptr,
                                   Layout2<L, E>::rows_total(),
                                   (WG / TPT) * ((1 << L) / 2 + 1) * 16 + (WG / TPT) * Layout2<L, E>::region() * 8});
    }
}

template <int LOG2N, int LOG2EPT, int WG>
void add_signs()
{
    add_st2<LOG2N, LOG2EPT, WG, -1>();
    add_st2<LOG2N, LOG2EPT, WG, +1>();
    add_one<LOG2N, LOG2EPT, WG, -1>();
    add_one<LOG2N, LOG2EPT, WG, +1>();
    add_st<LOG2N, LOG2EPT, WG, -1>();
    add_st<LOG2N, LOG2EPT, WG, +1>();
    // kinds: 1 = TW0 PF0, 2 = TW1 PF0, 3 = TW0 PF1, 4 = TW1 PF1; 5..8 the same
    // with wave-local exchanges (transforms of at most 64 threads)
    add_v2<LOG2N, LOG2EPT, WG, -1, 0, 0>();
    add_v2<LOG2N, LOG2EPT, WG, +1, 0, 0>();
    add_v2<LOG2N, LOG2EPT, WG, -1, 1, 0>();
    add_v2<LOG2N, LOG2EPT, WG, +1, 1, 0>();
    add_v2<LOG2N, LOG2EPT, WG, -1, 0, 1>();
    add_v2<LOG2N, LOG2EPT, WG, +1, 0, 1>();
    add_v2<LOG2N, LOG2EPT, WG, -1, 1, 1>();
    add_v2<LOG2N, LOG2EPT, WG, +1, 1, 1>();
}

template <int LOG2N, int LOG2EPT>
void add_wgs()
{
    add_signs<LOG2N, LOG2EPT, 64>();
    add_signs<LOG2N, LOG2EPT, 128>();
    add_signs<LOG2N, LOG2EPT, 256>();
    add_signs<LOG2N, LOG2EPT, 512>();
    add_signs<LOG2N, LOG2EPT, 1024>();
}

struct Registrar {
    Registrar()
    {
        add_wgs<MIFFT_LOG2N, 1>();
        add_wgs<MIFFT_LOG2N, 2>();
        add_wgs<MIFFT_LOG2N, 3>();
        add_wgs<MIFFT_LOG2N, 4>();
    }
};
Registrar registrar;

}  // namespace
}  // namespace mifft
