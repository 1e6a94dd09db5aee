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
#include <hip/hip_runtime.h>
#include <stdint.h>

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
    static constexpr int log2r(int p) { return (REM && p == 0) ? REM : LOG2EPT; }
    static constexpr int log2ns(int p)
    {
        return p == 0 ? 0 : (REM ? REM + (p - 1) * LOG2EPT : p * LOG2EPT);
    }
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
    using SC = Sched<LOG2N, LOG2EPT>;
    constexpr int LR = SC::log2r(P);
    constexpr int LNS = SC::log2ns(P), NS = 1 << LNS;
    const int j = t + q * SC::TPT;
    const int k = j & (NS - 1);
    return ((j >> LNS) << (LNS + LR)) + k + r * NS;
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

}  // namespace mifft
