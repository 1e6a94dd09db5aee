// Device building blocks of the FP32 Stockham FFT for gfx950 (CDNA4).
//
// Paper section "Fast Fourier Transform": a length-N DFT (Eq. (dft)) of
// power-of-two length is evaluated breadth-first, one Cooley-Tukey stage
// after another, with higher radices (the paper names radix-4, -8 and -16)
// so that there are fewer stages.  Here every stage is a Stockham
// (self-sorting) pass: each thread holds EPT complex values in VGPRs,
// applies the inter-stage twiddles of Eq. (radix2) generalised to radix R,
// runs R-point DFTs in registers and exchanges through LDS, so input and
// output are both in natural order and nothing is bit-reversed.
//
// Index bookkeeping of one pass (radix R, NS = product of the radices of
// the passes already done, butterfly j in [0, N/R)):
//   reads   x[j + r N/R],  r < R
//   k     = j mod NS
//   y_r  <- x[j + r N/R] * w_{NS R}^{r k}          (twiddle, skipped if NS = 1)
//   Y     = DFT_R(y)                               (in registers)
//   writes Y_r to  (j - k) R + k + r NS
// With this, thread t always holds elements t + m N/EPT (m < EPT) at the
// start of every pass: a contiguous, coalesced pattern in HBM and in LDS.
#pragma once

#include <utility>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "index_maps.hpp"

namespace mifft {

struct alignas(8) cf {
    float x, y;
};

__device__ __forceinline__ cf cadd(cf a, cf b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cf csub(cf a, cf b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cf cmul(cf a, cf b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ cf cscale(cf a, float s) { return {a.x * s, a.y * s}; }

// a * (S i), S = +-1: the quarter-period rotation of Eq. (twiddle) is a swap
// and a negation, no multiply.
template <int S>
__device__ __forceinline__ cf mul_si(cf a)
{
    if constexpr (S > 0)
        return {-a.y, a.x};
    else
        return {a.y, -a.x};
}

// cos(2 pi e / 16) and sin(2 pi e / 16), e = 0..15.
constexpr float kCos16[16] = {
    1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
    0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
    -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f,
    0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f};
constexpr float kSin16[16] = {
    0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f,
    1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
    0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
    -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f};
constexpr float kRsqrt2 = 0.70710678118654752f;

// a * exp(S 2 pi i E / 16) with E known at compile time: multiples of 1/4
// turn are swaps/negations, odd multiples of 1/8 turn cost two multiplies.
template <int S, int E>
__device__ __forceinline__ cf rot16(cf a)
{
    constexpr int e = ((E % 16) + 16) % 16;
    if constexpr (e == 0) {
        return a;
    } else if constexpr (e == 4) {
        return mul_si<S>(a);
    } else if constexpr (e == 8) {
        return {-a.x, -a.y};
    } else if constexpr (e == 12) {
        return mul_si<-S>(a);
    } else if constexpr (e == 2 || e == 6 || e == 10 || e == 14) {
        // (c + S i s) with |c| = |s| = 1/sqrt2
        constexpr float c = kCos16[e] > 0 ? 1.0f : -1.0f;
        constexpr float s = (kSin16[e] > 0 ? 1.0f : -1.0f) * (float)S;
        return {kRsqrt2 * (c * a.x - s * a.y), kRsqrt2 * (c * a.y + s * a.x)};
    } else {
        constexpr float c = kCos16[e];
        constexpr float s = kSin16[e] * (float)S;
        return {c * a.x - s * a.y, c * a.y + s * a.x};
    }
}

// ---------------------------------------------------------------- R-point DFTs
// In place, natural order in and out: X_k = sum_n x_n exp(S 2 pi i k n / R).

template <int S>
__device__ __forceinline__ void dft2(cf& a, cf& b)
{
    const cf t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <int S>
__device__ __forceinline__ void dft4(cf& a0, cf& a1, cf& a2, cf& a3)
{
    const cf t0 = cadd(a0, a2), t1 = csub(a0, a2);
    const cf t2 = cadd(a1, a3), t3 = mul_si<S>(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

// radix-8 = two radix-4 DFTs on the even and odd samples, then one radix-2
// stage with the twiddles exp(S 2 pi i k / 8) (Eq. (radix2) with N = 8).
template <int S>
__device__ __forceinline__ void dft8(cf (&x)[8])
{
    cf e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
    cf o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
    dft4<S>(e0, e1, e2, e3);
    dft4<S>(o0, o1, o2, o3);
    o1 = rot16<S, 2>(o1);
    o2 = rot16<S, 4>(o2);
    o3 = rot16<S, 6>(o3);
    x[0] = cadd(e0, o0);
    x[4] = csub(e0, o0);
    x[1] = cadd(e1, o1);
    x[5] = csub(e1, o1);
    x[2] = cadd(e2, o2);
    x[6] = csub(e2, o2);
    x[3] = cadd(e3, o3);
    x[7] = csub(e3, o3);
}

template <int S, int N2>
__device__ __forceinline__ void rot_row16(cf (&y)[16])
{
    y[4 * N2 + 1] = rot16<S, N2 * 1>(y[4 * N2 + 1]);
    y[4 * N2 + 2] = rot16<S, N2 * 2>(y[4 * N2 + 2]);
    y[4 * N2 + 3] = rot16<S, N2 * 3>(y[4 * N2 + 3]);
}

// radix-16 as 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2.
//   Y[n2][k1] = DFT4 over n1 of x[4 n1 + n2]
//   Y[n2][k1] *= exp(S 2 pi i n2 k1 / 16)
//   X[k1 + 4 k2] = DFT4 over n2 of Y[n2][k1]
template <int S>
__device__ __forceinline__ void dft16(cf (&x)[16])
{
    cf y[16];
#pragma unroll
    for (int n2 = 0; n2 < 4; n2++) {
        cf a0 = x[n2], a1 = x[4 + n2], a2 = x[8 + n2], a3 = x[12 + n2];
        dft4<S>(a0, a1, a2, a3);
        y[4 * n2 + 0] = a0;
        y[4 * n2 + 1] = a1;
        y[4 * n2 + 2] = a2;
        y[4 * n2 + 3] = a3;
    }
    rot_row16<S, 1>(y);
    rot_row16<S, 2>(y);
    rot_row16<S, 3>(y);
#pragma unroll
    for (int k1 = 0; k1 < 4; k1++) {
        cf a0 = y[k1], a1 = y[4 + k1], a2 = y[8 + k1], a3 = y[12 + k1];
        dft4<S>(a0, a1, a2, a3);
        x[k1] = a0;
        x[k1 + 4] = a1;
        x[k1 + 8] = a2;
        x[k1 + 12] = a3;
    }
}

// DFT_R on the R values v[Q0 + r * QS], r < R, of a thread's register array.
template <int R, int S, int QS, int EPT>
__device__ __forceinline__ void dft_strided(cf (&v)[EPT], int q0)
{
    cf x[R];
#pragma unroll
    for (int r = 0; r < R; r++)
        x[r] = v[q0 + r * QS];
    if constexpr (R == 2) {
        dft2<S>(x[0], x[1]);
    } else if constexpr (R == 4) {
        dft4<S>(x[0], x[1], x[2], x[3]);
    } else if constexpr (R == 8) {
        dft8<S>(x);
    } else {
        static_assert(R == 16, "radix must be 2, 4, 8 or 16");
        dft16<S>(x);
    }
#pragma unroll
    for (int r = 0; r < R; r++)
        v[q0 + r * QS] = x[r];
}

// ---------------------------------------------------------------- schedule
// log2 N = a * log2 EPT + rem: one radix-2^rem pass first (twiddle-free,
// NS = 1), then passes of radix EPT.
template <int LOG2N, int LOG2EPT>
struct Sched {
    static constexpr int N = 1 << LOG2N;
    static constexpr int EPT = 1 << LOG2EPT;
    static constexpr int TPT = N / EPT;  // threads per transform
    static constexpr int REM = LOG2N % LOG2EPT;
    static constexpr int NP = LOG2N / LOG2EPT + (REM ? 1 : 0);
    static constexpr int log2r(int p) { return idx::sched_log2r(LOG2N, LOG2EPT, p); }
    static constexpr int log2ns(int p) { return idx::sched_log2ns(LOG2N, LOG2EPT, p); }
    static_assert(LOG2EPT >= 1 && LOG2EPT <= 4, "EPT must be 2..16");
    static_assert(LOG2EPT <= LOG2N, "EPT must not exceed N");
};

// LDS swizzle: XOR of bits [5, 11) into bits [0, 6).  A bijection inside each
// aligned 64-word block, so contiguous reads stay conflict-free across the 64
// banks, while the strided writes of the early passes spread over banks.
__device__ __forceinline__ int swz(int i) { return i ^ ((i >> 5) & 63); }

// Twiddle of pass p for butterfly j, input r: exp(S 2 pi i r k / (NS R)),
// read from the 2048-entry table tw[m] = exp(-2 pi i m / 2048).
template <int S>
__device__ __forceinline__ cf twiddle(const cf* __restrict__ tw, int idx)
{
    cf w = tw[idx];
    if constexpr (S > 0)
        w.y = -w.y;
    return w;
}

// One transform-set pass: twiddle + DFT_R on the registers of thread t.
template <int LOG2N, int LOG2EPT, int S, int P>
__device__ __forceinline__ void pass_compute(cf (&v)[1 << LOG2EPT], int t, const cf* __restrict__ tw)
{
    using SC = Sched<LOG2N, LOG2EPT>;
    constexpr int LR = SC::log2r(P), R = 1 << LR;
    constexpr int LNS = SC::log2ns(P), NS = 1 << LNS;
    constexpr int EPT = SC::EPT, TPT = SC::TPT, Q = EPT / R;
    if constexpr (NS > 1) {
        constexpr int SHIFT = 11 - LNS - LR;
        static_assert(SHIFT >= 0, "the 2048-entry table resolves twiddles of passes up to NS R = 2048");
#pragma unroll
        for (int q = 0; q < Q; q++) {
            const int j = t + q * TPT;
            const int k = j & (NS - 1);
#pragma unroll
            for (int r = 1; r < R; r++)
                v[q + r * Q] = cmul(v[q + r * Q], twiddle<S>(tw, (r * k) << SHIFT));
        }
    }
#pragma unroll
    for (int q = 0; q < Q; q++)
        dft_strided<R, S, Q, EPT>(v, q);
}

// Destination index of output r of butterfly q of thread t in pass P.
template <int LOG2N, int LOG2EPT, int P>
__device__ __forceinline__ int pass_dst(int t, int q, int r)
{
    return idx::stockham_dst(LOG2N, LOG2EPT, P, t + q * Sched<LOG2N, LOG2EPT>::TPT, r);
}

// All passes of one transform held by a set of TPT threads.
//   v      : EPT values of thread t, loaded as x[t + m TPT]
//   lre/lim: this transform's LDS planes (N floats each, swizzled)
// On return v holds X[t + m TPT] (natural order) ready for the store.
// Every thread of the workgroup must call this (it contains barriers).
template <int LOG2N, int LOG2EPT, int S, int P = 0>
__device__ __forceinline__ void run_passes(cf (&v)[1 << LOG2EPT], int t, const cf* __restrict__ tw,
                                           float* lre, float* lim)
{
    using SC = Sched<LOG2N, LOG2EPT>;
    constexpr int EPT = SC::EPT, TPT = SC::TPT;
    pass_compute<LOG2N, LOG2EPT, S, P>(v, t, tw);
    if constexpr (P + 1 < SC::NP) {
        constexpr int LR = SC::log2r(P), R = 1 << LR, Q = EPT / R;
        if constexpr (P > 0)
            __syncthreads();  // everyone has read the previous exchange
#pragma unroll
        for (int q = 0; q < Q; q++)
#pragma unroll
            for (int r = 0; r < R; r++) {
                const int d = swz(pass_dst<LOG2N, LOG2EPT, P>(t, q, r));
                lre[d] = v[q + r * Q].x;
                lim[d] = v[q + r * Q].y;
            }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < EPT; m++) {
            const int s = swz(t + m * TPT);
            v[m] = cf{lre[s], lim[s]};
        }
        run_passes<LOG2N, LOG2EPT, S, P + 1>(v, t, tw, lre, lim);
    }
}

// ======================================================================
// Persistent variant ("v2") building blocks.
//
// LDS exchanges use AoS complex values and the padding pad(d) = d + (d >> B)
// (one spare slot every 2^B elements), with B chosen per exchange so that
// (a) both the writes of pass P and the reads of pass P+1 stay affine in the
// compile-time indices -- every address is one per-thread base plus an
// immediate offset, no per-element index arithmetic -- and (b) the modelled
// bank conflicts of the 64-bank LDS are lowest among such B.  B = 0 means
// no padding.
using idx::pad_bits;
using idx::pad_is_affine;

template <int B>
__device__ __forceinline__ int pad(int d)
{
    return idx::pad_index(B, d);
}

template <int L, int E>
struct Layout2 {
    using SC = Sched<L, E>;
    static constexpr int N = SC::N;
    // LDS elements per transform: the largest padded size over the exchanges
    static constexpr int region() { return idx::region(L, E); }
    // twiddle rows: for each pass P >= 1 (NS > 1), NS rows of EPT entries
    // w_{NS R}^{r k}, r < R = EPT (entry 0 is 1).
    static constexpr int rows_offset(int P) { return idx::rows_offset(L, E, P); }
    static constexpr int rows_total() { return idx::rows_total(L, E); }
};

// Twiddles of pass P for thread t, read as EPT/2 16-byte loads of one row.
// PAD > 0: the table is a copy whose rows of EPT values are padded to
// EPT + PAD (copy_rows_padded), for LDS: with PAD = 2 the 16-byte reads of
// 16 consecutive rows cover the 64 banks once (rows 144 bytes apart).
template <int L, int E, int S, int P, int PAD = 0>
__device__ __forceinline__ void load_row(cf (&w)[1 << E], const cf* __restrict__ rows, int t)
{
    using SC = Sched<L, E>;
    constexpr int EPT = SC::EPT, NS = 1 << SC::log2ns(P), RS = EPT + PAD;
    static_assert(SC::log2r(P) == E, "twiddled passes have radix EPT");
    static_assert(PAD % 2 == 0, "rows stay 16-byte aligned");
    if constexpr (idx::rows_entry_major(L)) {
        // entry r of row k at rows_offset(P) + r NS + k: consecutive lanes,
        // consecutive addresses
        static_assert(PAD == 0, "entry-major rows are read from the table");
        const cf* base = rows + Layout2<L, E>::rows_offset(P) + (t & (NS - 1));
#pragma unroll
        for (int r = 0; r < EPT; r++) {
            const cf q = base[r * NS];
            w[r] = cf{q.x, S > 0 ? -q.y : q.y};
        }
        return;
    }
    const float4* r4 =
        reinterpret_cast<const float4*>(rows + Layout2<L, E>::rows_offset(P) / EPT * RS + (t & (NS - 1)) * RS);
#pragma unroll
    for (int i = 0; i < EPT / 2; i++) {
        const float4 q = r4[i];
        w[2 * i] = cf{q.x, S > 0 ? -q.y : q.y};
        w[2 * i + 1] = cf{q.z, S > 0 ? -q.w : q.w};
    }
}

// Copies the twiddle-row table `src` (rows of EPT values) to `dst` with each
// row padded to EPT + PAD values, threads tid, tid + nthreads, ... .
template <int L, int E, int PAD>
__device__ __forceinline__ void copy_rows_padded(cf* dst, const cf* __restrict__ src, int tid, int nthreads)
{
    static_assert(!idx::rows_entry_major(L), "row-major tables only");
    constexpr int EPT = 1 << E, TOT = Layout2<L, E>::rows_total();
    for (int i = tid; i < TOT; i += nthreads)
        dst[i / EPT * (EPT + PAD) + i % EPT] = src[i];
}

template <int L, int E, int PAD>
__host__ __device__ constexpr int padded_rows_total()
{
    return Layout2<L, E>::rows_total() / (1 << E) * ((1 << E) + PAD);
}

// Twiddle + butterflies of pass P given the row values w (ignored if NS = 1).
template <int L, int E, int S, int P>
__device__ __forceinline__ void pass_compute2(cf (&v)[1 << E], const cf (&w)[1 << E])
{
    using SC = Sched<L, E>;
    constexpr int LR = SC::log2r(P), R = 1 << LR, NS = 1 << SC::log2ns(P), Q = SC::EPT / R;
    if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; r++)
            v[r] = cmul(v[r], w[r]);
    }
#pragma unroll
    for (int q = 0; q < Q; q++)
        dft_strided<R, S, Q, SC::EPT>(v, q);
}

// Orders LDS accesses between the threads that share a transform.  When a
// transform's threads all sit in one wavefront (WAVE), its LDS region is
// private to that wavefront and LDS instructions of a wavefront execute in
// issue order, so only compiler reordering must be prevented: no s_barrier.
// Otherwise a workgroup barrier.
template <bool WAVE>
__device__ __forceinline__ void lds_sync()
{
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Exchange after pass P through this transform's LDS region `lds`.
template <int L, int E, int P, bool WAVE>
__device__ __forceinline__ void exchange2(cf (&v)[1 << E], int t, cf* lds)
{
    using SC = Sched<L, E>;
    constexpr int LR = SC::log2r(P), R = 1 << LR, LNS = SC::log2ns(P), NS = 1 << LNS;
    constexpr int EPT = SC::EPT, Q = EPT / R;
    constexpr idx::Strides ST = idx::exchange_strides(L, E, P);
    constexpr int B = ST.B, DR = ST.DR, DQ = ST.DQ, DM = ST.DM;
    static_assert(pad_is_affine(L, E, P, B), "padding must keep addresses affine");
    // base: r = 0, q = 0
    const int k = t & (NS - 1);
    const int d0 = ((t >> LNS) << (LNS + LR)) + k;
    cf* wb = lds + pad<B>(d0);
#pragma unroll
    for (int q = 0; q < Q; q++)
#pragma unroll
        for (int r = 0; r < R; r++)
            wb[q * DQ + r * DR] = v[q + r * Q];
    lds_sync<WAVE>();
    const cf* rb = lds + pad<B>(t);
#pragma unroll
    for (int m = 0; m < EPT; m++)
        v[m] = rb[m * DM];
}

// ---------------------------------------------------------------- global data access
typedef float v2f __attribute__((ext_vector_type(2)));
// Types for HBM data: declared 4-byte aligned, so buffers need only be
// aligned to their element (complex64: 8 bytes; float32 reals and 16-bit
// (re, im) pairs: 4 bytes).  gfx950 serves dword-aligned multi-dword global
// accesses in hardware, and the compiler still emits one dwordx2 / dwordx4
// instruction for each.
typedef float gv2 __attribute__((ext_vector_type(2), aligned(4)));
typedef float gv4 __attribute__((ext_vector_type(4), aligned(4)));
typedef uint32_t gu4 __attribute__((ext_vector_type(4), aligned(4)));

// Transform data is streamed: read once, written once.  Nontemporal
// accesses (NT) keep it from displacing the twiddle tables in the caches
// and measured 5-7% faster at N = 2048 on MI355X -- but only when every
// wave-wide load/store instruction covers whole 128-byte lines.  When a
// line is split across instructions (runs of fewer than 16 consecutive
// complex values per transform) the streamed line is fetched again for the
// second instruction, and plain accesses are much faster.
template <int N, int TPT>
constexpr bool stream_nt()
{
    return TPT >= 16 || (TPT == 1 && N == 2);
}

template <bool NT>
__device__ __forceinline__ cf ld_data(const char* p)
{
    const gv2* q = reinterpret_cast<const gv2*>(p);
    gv2 v;
    if constexpr (NT)
        v = __builtin_nontemporal_load(q);
    else
        v = *q;
    return cf{v.x, v.y};
}

template <bool NT>
__device__ __forceinline__ void st_data(char* p, cf v)
{
    gv2 w;
    w.x = v.x;
    w.y = v.y;
    gv2* q = reinterpret_cast<gv2*>(p);
    if constexpr (NT)
        __builtin_nontemporal_store(w, q);
    else
        *q = w;
}

// One complex value of HBM data at any 4-byte-aligned address.
__device__ __forceinline__ cf ld_c(const cf* p) { return ld_data<false>(reinterpret_cast<const char*>(p)); }
__device__ __forceinline__ void st_c(cf* p, cf v) { st_data<false>(reinterpret_cast<char*>(p), v); }

template <int L, int E, int TPB>
__device__ __forceinline__ void load_group(cf (&v)[1 << E], const cf* __restrict__ in, int64_t g, int64_t batch,
                                           int tb, unsigned toff8)
{
    using SC = Sched<L, E>;
    constexpr int N = SC::N, EPT = SC::EPT, TPT = SC::TPT;
    constexpr bool NT = stream_nt<N, TPT>();
    const int64_t first = g * TPB;
    const char* gb = reinterpret_cast<const char*>(in + first * N);
    unsigned off = toff8;
    if constexpr (TPB > 1) {
        // Threads of a transform past the end of the batch (last group
        // only) read the batch's last transform instead: every thread
        // issues the same loads, with no branch around them, and those
        // results are never stored.
        const int64_t last = batch - 1 - first;
        off = first + tb < batch ? toff8 : (unsigned)(last * N + (toff8 / 8u) % (unsigned)TPT) * 8u;
    }
#pragma unroll
    for (int m = 0; m < EPT; m++)
        v[m] = ld_data<NT>(gb + (off + (unsigned)(m * TPT * 8)));
}

// Elements m in [K EPT/NK, (K+1) EPT/NK) of a group load (slice K of NK),
// with the same threads-past-the-end rule as load_group.
template <int L, int E, int TPB, int K, int NK>
__device__ __forceinline__ void load_group_part(cf (&v)[1 << E], const cf* __restrict__ in, int64_t g,
                                                int64_t batch, int tb, unsigned toff8)
{
    using SC = Sched<L, E>;
    constexpr int N = SC::N, EPT = SC::EPT, TPT = SC::TPT;
    constexpr bool NT = stream_nt<N, TPT>();
    constexpr int M0 = K * EPT / NK, M1 = (K + 1) * EPT / NK;
    const int64_t first = g * TPB;
    const char* gb = reinterpret_cast<const char*>(in + first * N);
    unsigned off = toff8;
    if constexpr (TPB > 1) {
        const int64_t last = batch - 1 - first;
        off = first + tb < batch ? toff8 : (unsigned)(last * N + (toff8 / 8u) % (unsigned)TPT) * 8u;
    }
#pragma unroll
    for (int m = M0; m < M1; m++)
        v[m] = ld_data<NT>(gb + (off + (unsigned)(m * TPT * 8)));
}

template <int L, int E, int TPB>
__device__ __forceinline__ void store_group(const cf (&v)[1 << E], cf* __restrict__ out, int64_t g, int64_t batch,
                                            int tb, unsigned toff8, float scale)
{
    using SC = Sched<L, E>;
    constexpr int N = SC::N, EPT = SC::EPT, TPT = SC::TPT;
    constexpr bool NT = stream_nt<N, TPT>();
    const int64_t first = g * TPB;
    char* gb = reinterpret_cast<char*>(out + first * N);
    // One transform per group: every group a kernel stores (g < batch) is
    // whole, and the stores carry no branch.  A branch around them would make
    // the wait counter's bookkeeping after it allow for the stores not having
    // been issued, so a later wait for a load issued before them would wait
    // for the stores as well.
    if (TPB == 1 || first + TPB <= batch || first + tb < batch) {
#pragma unroll
        for (int m = 0; m < EPT; m++)
            st_data<NT>(gb + (toff8 + (unsigned)(m * TPT * 8)), cscale(v[m], scale));
    }
}

// ---------------------------------------------------------------- pass runner
template <int L, int E>
using TwRegs = cf[Sched<L, E>::NP][1 << E];

template <int L, int E, int S, int P = 0>
__device__ __forceinline__ void load_all_rows(TwRegs<L, E>& tws, const cf* __restrict__ rows, int t)
{
    if constexpr (P < Sched<L, E>::NP) {
        if constexpr (Sched<L, E>::log2ns(P) > 0)
            load_row<L, E, S, P>(tws[P], rows, t);
        load_all_rows<L, E, S, P + 1>(tws, rows, t);
    }
}

template <int L, int E, int S, int TW, bool WAVE, int P = 0, int PAD = 0>
__device__ __forceinline__ void run2(cf (&v)[1 << E], int t, const cf* __restrict__ rows,
                                     const TwRegs<L, E>& tws, cf* lds)
{
    using SC = Sched<L, E>;
    constexpr int EPT = SC::EPT;
    if constexpr (SC::log2ns(P) > 0) {
        if constexpr (TW == 0) {
            pass_compute2<L, E, S, P>(v, tws[P]);
        } else {
            cf w[EPT];
            load_row<L, E, S, P, PAD>(w, rows, t);
            pass_compute2<L, E, S, P>(v, w);
        }
    } else {
        pass_compute2<L, E, S, P>(v, tws[0]);
    }
    if constexpr (P + 1 < SC::NP) {
        if constexpr (P > 0)
            lds_sync<WAVE>();  // all reads of the previous exchange are done
        exchange2<L, E, P, WAVE>(v, t, lds);
        run2<L, E, S, TW, WAVE, P + 1, PAD>(v, t, rows, tws, lds);
    }
}

// run2 that also loads the next group (transform group `gn` of `in`) into
// `nx`, one slice before each pass, so a workgroup's loads reach HBM spread
// over its passes rather than in one burst per group.
template <int L, int E, int S, int TW, bool WAVE, int TPB, int P = 0, int PAD = 0>
__device__ __forceinline__ void run2_prefetch(cf (&v)[1 << E], int t, const cf* __restrict__ rows,
                                              const TwRegs<L, E>& tws, cf* lds, cf (&nx)[1 << E],
                                              const cf* __restrict__ in, int64_t gn, int64_t batch, int tb,
                                              unsigned toff8)
{
    using SC = Sched<L, E>;
    constexpr int EPT = SC::EPT;
    if constexpr (SC::log2ns(P) > 0) {
        if constexpr (TW == 0) {
            load_group_part<L, E, TPB, P, SC::NP>(nx, in, gn, batch, tb, toff8);
            pass_compute2<L, E, S, P>(v, tws[P]);
        } else {
            // The pass's twiddle row is read before the slice (read after
            // it, its wait would cover the slice as well), and the
            // scheduling barrier keeps both ahead of the pass's arithmetic.
            cf w[EPT];
            load_row<L, E, S, P, PAD>(w, rows, t);
            load_group_part<L, E, TPB, P, SC::NP>(nx, in, gn, batch, tb, toff8);
            __builtin_amdgcn_sched_barrier(0);
            pass_compute2<L, E, S, P>(v, w);
        }
    } else {
        load_group_part<L, E, TPB, P, SC::NP>(nx, in, gn, batch, tb, toff8);
        if constexpr (TW != 0)
            __builtin_amdgcn_sched_barrier(0);
        pass_compute2<L, E, S, P>(v, tws[0]);
    }
    if constexpr (P + 1 < SC::NP) {
        if constexpr (P > 0)
            lds_sync<WAVE>();  // all reads of the previous exchange are done
        exchange2<L, E, P, WAVE>(v, t, lds);
        run2_prefetch<L, E, S, TW, WAVE, TPB, P + 1, PAD>(v, t, rows, tws, lds, nx, in, gn, batch, tb, toff8);
    }
}

// run2 over workgroup-wide exchanges that calls slice(P) before pass P,
// after that pass's twiddle row is read: a caller's loads for its next tile,
// spread over the passes.  Passes P < K read their rows from `lrows`, a copy
// in LDS with the row padding PAD (copy_rows_padded, the first K passes'
// rows); later passes from `grows`, the table itself.  A wait for an LDS
// row covers none of the slices' global loads; a wait for a global row
// covers the slices issued before it.
template <int L, int E, int S, int PAD, int K, int P = 0, class F>
__device__ __forceinline__ void run2_slices(cf (&v)[1 << E], int t, const cf* lrows, const cf* __restrict__ grows,
                                            cf* lds, F& slice)
{
    using SC = Sched<L, E>;
    cf w[SC::EPT];
    if constexpr (SC::log2ns(P) > 0) {
        if constexpr (P < K)
            load_row<L, E, S, P, PAD>(w, lrows, t);
        else
            load_row<L, E, S, P, 0>(w, grows, t);
    }
    slice(std::integral_constant<int, P>{});
    pass_compute2<L, E, S, P>(v, w);
    if constexpr (P + 1 < SC::NP) {
        if constexpr (P > 0)
            lds_sync<false>();  // all reads of the previous exchange are done
        exchange2<L, E, P, false>(v, t, lds);
        run2_slices<L, E, S, PAD, K, P + 1>(v, t, lrows, grows, lds, slice);
    }
}

// Leading passes whose twiddle rows, padded by PAD, fit in `bytes` of LDS.
template <int L, int E, int PAD>
__host__ __device__ constexpr int rows_prefix_passes(int bytes)
{
    int k = 0;
    while (k < Sched<L, E>::NP && Layout2<L, E>::rows_offset(k + 1) / (1 << E) * ((1 << E) + PAD) * 8 <= bytes)
        k++;
    return k;
}

// Entries (float2) of the padded LDS copy of the first K passes' rows.
template <int L, int E, int PAD>
__host__ __device__ constexpr int padded_rows_prefix(int K)
{
    return Layout2<L, E>::rows_offset(K) / (1 << E) * ((1 << E) + PAD);
}

// Copies the first K passes' rows of `src` to `dst`, padded as above.
template <int L, int E, int PAD, int K>
__device__ __forceinline__ void copy_rows_prefix_padded(cf* dst, const cf* __restrict__ src, int tid, int nthreads)
{
    static_assert(!idx::rows_entry_major(L), "row-major tables only");
    constexpr int EPT = 1 << E, TOT = Layout2<L, E>::rows_offset(K);
    for (int i = tid; i < TOT; i += nthreads)
        dst[i / EPT * (EPT + PAD) + i % EPT] = src[i];
}

}  // namespace mifft
