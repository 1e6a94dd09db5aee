// Real-input transforms (FFT_R32), one translation unit per half length:
// compiled with -DMIFFT_LOG2M=<0..14>, M = n/2.
//
// A real sequence x of even length n is read as the M complex values
// z_j = x_{2j} + i x_{2j+1} (the same bytes), so one length-M complex DFT
// carries the work.  With Z = DFT_M(z), the even/odd split of the radix-2
// step, Eq. (radix2), gives the spectrum of x (w = w_n = exp(-2 pi i / n)):
//   E_k = (Z_k + conj Z_{M-k}) / 2            (DFT_M of x_{2j})
//   O_k = (Z_k - conj Z_{M-k}) / (2i)         (DFT_M of x_{2j+1})
//   X_k = E_k + w^k O_k,   k = 0..M           (Z_M = Z_0)
// R2C (dir 0): load z, Stockham passes with sign -1, pair Z_k with Z_{M-k}
// through LDS, write X_0..X_M (n/2 + 1 bins per transform).
// C2R (dir 1) runs the same steps backwards from the bins X_0..X_M (the
// imaginary parts of X_0 and X_M are ignored: for a real sequence they are
// zero):
//   Z'_k = (X_k + conj X_{M-k}) + i conj(w^k) (X_k - conj X_{M-k})
// then the passes with sign +1 and x_{2j} = Re z_j, x_{2j+1} = Im z_j of
// z = sum_k Z'_k w_M^{-jk}, which is n times the inverse of Eq. (idft).
//
// Weights: R2C multiplies bins 0 and M by `we` and the others by `wi`; C2R
// multiplies Z'_0 (built from bins 0 and M) by `we` and Z'_k, 0 < k < M
// (built from two interior bins), by `wi`.  Plain transforms use (1, 1) and
// (1/n, 1/n); the adjoints are the other direction with (1, 1/2) for the
// adjoint of R2C and (1/n, 2/n) for the adjoint of C2R.
#include "device_fft.hpp"
#include "launch.hpp"
#include "real.hpp"

#ifndef MIFFT_LOG2M
#error "compile with -DMIFFT_LOG2M=<0..14>"
#endif

namespace mifft {
namespace {

// X_k from a = Z_k, b = Z_{M-k} and w = w_n^k.
__device__ __forceinline__ cf r2c_bin(cf a, cf b, cf w)
{
    const float sx = 0.5f * (a.x + b.x), sy = 0.5f * (a.y - b.y);  // (a + conj b) / 2
    const float dx = 0.5f * (a.y + b.y), dy = -0.5f * (a.x - b.x);  // (a - conj b) / (2i)
    return cf{sx + w.x * dx - w.y * dy, sy + w.x * dy + w.y * dx};
}

// Z'_k from a = X_k, b = X_{M-k} and w = w_n^k.
__device__ __forceinline__ cf c2r_pre(cf a, cf b, cf w)
{
    const float dx = a.x - b.x, dy = a.y + b.y;  // a - conj b
    return cf{a.x + b.x - w.x * dy + w.y * dx, a.y - b.y + w.x * dx + w.y * dy};
}

template <int L, int E, int WG>
struct RealShape {
    using SC = Sched<L, E>;
    static constexpr int M = SC::N, EPT = SC::EPT, TPT = SC::TPT, TPB = WG / TPT;
    static constexpr bool XCH = TPT > 1;  // the transform spans threads: LDS exchanges
    static constexpr int REG = XCH ? Layout2<L, E>::region() : 1;
};

// C2R input: bins k = t + m TPT of transform (g TPB + tb), plus bin M in
// thread 0 of the transform.  Transforms hold M + 1 bins each.
template <int L, int E, int WG>
__device__ __forceinline__ void load_bins(cf (&a)[1 << E], cf& aM, const cf* __restrict__ in, int64_t g,
                                          int64_t batch, int tb, int t)
{
    using RS = RealShape<L, E, WG>;
    constexpr int M = RS::M, TPT = RS::TPT;
    const int64_t first = g * RS::TPB;
    const char* ib = reinterpret_cast<const char*>(in + first * (M + 1));
    // Threads of a transform past the end of the batch re-read the batch's
    // last transform (never stored), and every thread reads bin M of its
    // transform: the loads are the same for every thread, with no branch
    // around them.
    const int64_t tr = first + tb < batch ? tb : batch - 1 - first;
    const unsigned o8 = (unsigned)(tr * (M + 1) + t) * 8u;
#pragma unroll
    for (int m = 0; m < RS::EPT; m++)
        a[m] = *reinterpret_cast<const cf*>(ib + (o8 + (unsigned)(m * TPT * 8)));
    const cf binM = *reinterpret_cast<const cf*>(ib + (unsigned)(tr * (M + 1) + M) * 8u);
    aM = t == 0 ? binM : cf{0.f, 0.f};
}

// One transform group, R2C: v holds z (loaded), leaves X in `out`.
template <int L, int E, int WG, int TW, bool WAVE>
__device__ __forceinline__ void r2c_group(cf (&v)[1 << E], cf* __restrict__ out, const cf* __restrict__ rows,
                                          const cf (&wv)[1 << E], const TwRegs<L, E>& tws, cf* my, int64_t g,
                                          int64_t batch, int tb, int t, float we, float wi)
{
    using RS = RealShape<L, E, WG>;
    constexpr int M = RS::M, EPT = RS::EPT, TPT = RS::TPT;
    run2<L, E, -1, TW, WAVE>(v, t, rows, tws, my);
    // v[m] = Z_k for k = t + m TPT; fetch Z_{M-k}
    cf zp[EPT];
    if constexpr (!RS::XCH) {
#pragma unroll
        for (int m = 0; m < EPT; m++)
            zp[m] = v[(M - m) & (M - 1)];
    } else {
        lds_sync<WAVE>();  // the last exchange is fully read
#pragma unroll
        for (int m = 0; m < EPT; m++)
            my[t + m * TPT] = v[m];
        lds_sync<WAVE>();
#pragma unroll
        for (int m = 0; m < EPT; m++)
            zp[m] = my[idx::real_partner(M, t + m * TPT)];
    }
    const int64_t first = g * RS::TPB;
    if (first + tb >= batch)
        return;
    char* ob = reinterpret_cast<char*>(out + first * (M + 1));
    const unsigned o8 = (unsigned)(tb * (M + 1) + t) * 8u;
#pragma unroll
    for (int m = 0; m < EPT; m++) {
        const cf x = r2c_bin(v[m], zp[m], wv[m]);
        const float s = (m == 0 && t == 0) ? we : wi;
        *reinterpret_cast<cf*>(ob + (o8 + (unsigned)(m * TPT * 8))) = cscale(x, s);
    }
    if (t == 0)  // X_M = E_0 - O_0
        *reinterpret_cast<cf*>(ob + (o8 + (unsigned)(M * 8))) = cf{(v[0].x - v[0].y) * we, 0.f};
}

// One transform group, C2R: v holds bins X_k (k = t + m TPT), vM bin M in
// thread 0; leaves x in `out`.
template <int L, int E, int WG, int TW, bool WAVE>
__device__ __forceinline__ void c2r_group(cf (&v)[1 << E], cf vM, cf* __restrict__ out, const cf* __restrict__ rows,
                                          const cf (&wv)[1 << E], const TwRegs<L, E>& tws, cf* my, int64_t g,
                                          int64_t batch, int tb, int t, float we, float wi)
{
    using RS = RealShape<L, E, WG>;
    constexpr int M = RS::M, EPT = RS::EPT, TPT = RS::TPT;
    cf bp[EPT];  // X_{M-k}
    if constexpr (!RS::XCH) {
        bp[0] = vM;
#pragma unroll
        for (int m = 1; m < EPT; m++)
            bp[m] = v[M - m];
    } else {
#pragma unroll
        for (int m = 0; m < EPT; m++)
            my[t + m * TPT] = v[m];
        lds_sync<WAVE>();
#pragma unroll
        for (int m = 0; m < EPT; m++)
            bp[m] = my[idx::real_partner(M, t + m * TPT)];
        if (t == 0)
            bp[0] = vM;
        lds_sync<WAVE>();  // partners read before the passes reuse LDS
    }
    if (t == 0) {
        v[0].y = 0.f;
        bp[0].y = 0.f;
    }
#pragma unroll
    for (int m = 0; m < EPT; m++) {
        const float s = (m == 0 && t == 0) ? we : wi;
        v[m] = cscale(c2r_pre(v[m], bp[m], wv[m]), s);
    }
    run2<L, E, +1, TW, WAVE>(v, t, rows, tws, my);
    store_group<L, E, RS::TPB>(v, out, g, batch, tb, (unsigned)(tb * M + t) * 8u, 1.f);
}

template <int L, int E, int WG, int DIR, int TW, int PF, bool WAVE>
__global__ __launch_bounds__(WG) void k_real(const cf* __restrict__ in, cf* __restrict__ out,
                                             const cf* __restrict__ rows, const cf* __restrict__ wn,
                                             int64_t batch, float we, float wi)
{
    using RS = RealShape<L, E, WG>;
    using SC = typename RS::SC;
    constexpr int M = RS::M, EPT = RS::EPT, TPT = RS::TPT, TPB = RS::TPB;
    static_assert(!WAVE || TPT <= 64, "wave-local exchanges need a transform inside one wavefront");
    __shared__ cf lds[RS::XCH ? TPB * RS::REG : 1];
    const int tid = threadIdx.x, tb = tid / TPT, t = tid % TPT;
    cf* my = lds + (RS::XCH ? tb * RS::REG : 0);
    const int64_t ngroups = (batch + TPB - 1) / TPB;
    int64_t g = blockIdx.x;
    if (g >= ngroups)
        return;
    cf tws[SC::NP][EPT];
#pragma unroll
    for (int p = 0; p < SC::NP; p++)
#pragma unroll
        for (int r = 0; r < EPT; r++)
            tws[p][r] = cf{1.f, 0.f};
    if constexpr (TW == 0 && RS::XCH)
        load_all_rows<L, E, DIR == 0 ? -1 : 1>(tws, rows, t);
    const unsigned toff8 = (unsigned)(tb * M + t) * 8u;
    cf a[EPT], b[EPT], aM = cf{0.f, 0.f}, bM = cf{0.f, 0.f};
    auto load = [&](cf(&v)[EPT], cf& vM, int64_t gg) {
        if constexpr (DIR == 0)
            load_group<L, E, TPB>(v, in, gg, batch, tb, toff8);
        else
            load_bins<L, E, WG>(v, vM, in, gg, batch, tb, t);
    };
    // The split's twiddles w[t + m TPT] are read at the top of each group,
    // before the next group's loads are issued: read after them, their
    // wait would cover the prefetch as well.
    cf wv[EPT];
    auto wload = [&]() {
#pragma unroll
        for (int m = 0; m < EPT; m++)
            wv[m] = wn[t + m * TPT];
        __builtin_amdgcn_sched_barrier(0);
    };
    auto process = [&](cf(&v)[EPT], cf vM, int64_t gg) {
        if constexpr (DIR == 0)
            r2c_group<L, E, WG, TW, WAVE>(v, out, rows, wv, tws, my, gg, batch, tb, t, we, wi);
        else
            c2r_group<L, E, WG, TW, WAVE>(v, vM, out, rows, wv, tws, my, gg, batch, tb, t, we, wi);
    };
    load(a, aM, g);
    if constexpr (!PF) {
        wload();
        process(a, aM, g);  // one group per workgroup (the grid covers every group)
        return;
    }
    // `left` groups follow the current one.  Inside the loop the next
    // group's load is unconditional (a conditional one makes the wait
    // before the current group's first use cover the prefetch too).
    const int64_t stride = gridDim.x;
    auto sync = [&]() {
        if constexpr (RS::XCH)
            lds_sync<WAVE>();  // LDS is reused by the next group
    };
    int64_t left = (ngroups - 1 - g) / stride;
    while (left >= 2) {
        wload();
        load(b, bM, g + stride);
        process(a, aM, g);
        g += stride;
        sync();
        wload();
        load(a, aM, g + stride);
        process(b, bM, g);
        g += stride;
        sync();
        left -= 2;
    }
    if (left == 1) {
        wload();
        load(b, bM, g + stride);
        process(a, aM, g);
        g += stride;
        sync();
        wload();
        process(b, bM, g);
    } else {
        wload();
        process(a, aM, g);
    }
}

// n = 2 (M = 1): one thread per transform, no passes.
template <int DIR>
__global__ __launch_bounds__(256) void k_real_n2(const cf* __restrict__ in, cf* __restrict__ out, int64_t batch,
                                                 float we, float wi)
{
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= batch)
        return;
    if constexpr (DIR == 0) {
        const cf z = in[b];  // (x0, x1)
        out[2 * b] = cf{(z.x + z.y) * we, 0.f};
        out[2 * b + 1] = cf{(z.x - z.y) * we, 0.f};
    } else {
        const float x0 = in[2 * b].x, x1 = in[2 * b + 1].x;
        out[b] = cf{(x0 + x1) * we, (x0 - x1) * we};
    }
}

template <int DIR>
hipError_t launch_real_n2(const void* in, void* out, const void*, const void*, int64_t batch, float we, float wi,
                          int64_t, hipStream_t stream)
{
    return launch_kernel((k_real_n2<DIR>), dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, stream,
                       static_cast<const cf*>(in), static_cast<cf*>(out), batch, we, wi);
}

template <int L, int E, int WG, int DIR, int TW, int PF, bool WAVE>
hipError_t launch_real(const void* in, void* out, const void* rows, const void* wn, int64_t batch, float we,
                       float wi, int64_t grid_limit, hipStream_t stream)
{
    constexpr int TPB = RealShape<L, E, WG>::TPB;
    int64_t grid = (batch + TPB - 1) / TPB;
    if (PF && grid_limit > 0 && grid > grid_limit)
        grid = grid_limit;
    return launch_kernel((k_real<L, E, WG, DIR, TW, PF, WAVE>), dim3((unsigned)grid), dim3(WG), 0, stream,
                       static_cast<const cf*>(in), static_cast<cf*>(out), static_cast<const cf*>(rows),
                       static_cast<const cf*>(wn), batch, we, wi);
}

template <int L, int E, int WG, int DIR, int TW, int PF, bool WAVE>
int occupancy_real()
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_real<L, E, WG, DIR, TW, PF, WAVE>, WG, 0) !=
        hipSuccess)
        return 0;
    return blocks;
}

// Menu: a whole half-length transform per thread for M <= 16 (kind 0);
// otherwise EPT 4, 8 or 16 with twiddle rows re-read and one group per
// workgroup (kind 2) or kept in registers with a persistent, prefetching
// loop (kind 3), plus their wavefront-local forms (6, 7) when a transform
// spans at most 64 threads.  WG <= 256 and LDS <= 64 KiB up to M = 2048;
// above, one transform per workgroup of up to 1024 threads, LDS <= 160 KiB.
template <int L, int E, int WG>
constexpr bool valid_real()
{
    if constexpr (E > L || E < 1 || E > 4) {
        return false;
    } else if constexpr (E == L) {
        return L <= 4;  // kind 0
    } else if constexpr (E < 2) {
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

template <int L, int E, int WG, int DIR, int TW, int PF, bool WAVE>
void add_real_kind(int kind)
{
    constexpr int TPT = (1 << L) >> E;
    constexpr int rows = TPT > 1 ? Layout2<L, E>::rows_total() : 0;
    constexpr int lds = TPT > 1 ? (WG / TPT) * Layout2<L, E>::region() * 8 : 0;
    register_real(KernelReal{L, E, WG, DIR, kind, &launch_real<L, E, WG, DIR, TW, PF, WAVE>,
                             &occupancy_real<L, E, WG, DIR, TW, PF, WAVE>, rows, lds});
}

template <int L, int E, int WG, int DIR>
void add_real()
{
    if constexpr (valid_real<L, E, WG>()) {
        constexpr int TPT = (1 << L) >> E;
        if constexpr (TPT == 1) {
            add_real_kind<L, E, WG, DIR, 1, 0, false>(0);
        } else {
            add_real_kind<L, E, WG, DIR, 1, 0, false>(2);
            add_real_kind<L, E, WG, DIR, 0, 1, false>(3);
            if constexpr (TPT <= 64) {
                add_real_kind<L, E, WG, DIR, 1, 0, true>(6);
                add_real_kind<L, E, WG, DIR, 0, 1, true>(7);
            }
        }
    }
}

template <int L, int E>
void add_real_wgs()
{
    if constexpr (L > 11) {
        add_real<L, E, ((1 << L) >> E), 0>();
        add_real<L, E, ((1 << L) >> E), 1>();
    } else {
        add_real<L, E, 64, 0>();
        add_real<L, E, 64, 1>();
        add_real<L, E, 128, 0>();
        add_real<L, E, 128, 1>();
        add_real<L, E, 256, 0>();
        add_real<L, E, 256, 1>();
    }
}

struct RealRegistrar {
    RealRegistrar()
    {
        constexpr int L = MIFFT_LOG2M;
        if constexpr (L == 0) {
            register_real(KernelReal{0, 0, 256, 0, 0, &launch_real_n2<0>, nullptr, 0, 0});
            register_real(KernelReal{0, 0, 256, 1, 0, &launch_real_n2<1>, nullptr, 0, 0});
        } else {
            add_real_wgs<L, 1>();
            add_real_wgs<L, 2>();
            add_real_wgs<L, 3>();
            add_real_wgs<L, 4>();
        }
    }
};
RealRegistrar real_registrar;

}  // namespace
}  // namespace mifft
