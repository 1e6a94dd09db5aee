// Twiddle table: tw[m] = exp(-2 pi i m / 2048), m < 2048, stored as FP32.
//
// The paper's twiddles w_N^k (Eq. (dft)) come from the device's own sin/cos
// (section "Portability and Precision").  Here they are generated once per
// plan on the GPU in FP64 with sincospi, rounded once to FP32; this is the
// only FP64 arithmetic in the library.  Every w_N^k with N <= 2048 is
// tw[k * 2048 / N].
//
// Symmetry is enforced so that the table is exact where the circle is:
// angles are folded into the first octant [0, pi/4], evaluated there, and
// unfolded with the swaps/negations of the quarter-period identities of
// Eq. (twiddle).  Hence w^{m + 512} = -i w^m holds bit for bit and the
// points at multiples of 1/8 turn are exact (to FP32 rounding of 1/sqrt 2).
#include <hip/hip_runtime.h>
#include "index_maps.hpp"
#include "launch.hpp"
#include <stdint.h>

namespace mifft {

__global__ void k_twiddle_2048(float2* __restrict__ tw)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= 2048)
        return;
    const int quad = m >> 9;     // quarter turn index (512 entries per quarter)
    const int j = m & 511;       // position inside the quarter
    // angle inside the quarter folded to [0, 1/8 turn]
    double c, s;
    if (j <= 256) {
        sincospi((double)j / 1024.0, &s, &c);
    } else {
        double c2, s2;
        sincospi((double)(512 - j) / 1024.0, &s2, &c2);
        c = s2;
        s = c2;
    }
    // rotate by quad quarter turns: (c, s) -> (-s, c)
    double cr = c, sr = s;
    if (quad == 1) {
        cr = -s;
        sr = c;
    } else if (quad == 2) {
        cr = -c;
        sr = -s;
    } else if (quad == 3) {
        cr = s;
        sr = -c;
    }
    // exp(-i theta) = cos theta - i sin theta
    tw[m] = float2{(float)cr, (float)(-sr)};
}

hipError_t launch_twiddle_2048(void* tw, hipStream_t stream)
{
    return launch_kernel(k_twiddle_2048, dim3(8), dim3(256), 0, stream, static_cast<float2*>(tw));
}

}  // namespace mifft

namespace mifft {

// Per-pass twiddle rows of a (log2 N, log2 EPT) Stockham schedule: for each
// pass with NS > 1 (radix EPT), NS rows of EPT entries, row k holding
// w_M^{r k}, M = NS EPT, r < EPT.  When M <= 2048 the entry is the copy
// tw[(r k) * 2048 / M] of the 2048-entry table, so every kernel family uses
// identical twiddles; for longer transforms (M > 2048, which the table does
// not resolve) it is evaluated here in FP64 with sincospi and rounded once.
__global__ void k_twiddle_rows(const float2* __restrict__ tw, float2* __restrict__ rows, int L, int E, int total)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total)
        return;
    const idx::RowEntry w = idx::twiddle_row_entry(L, E, i);
    if (w.pass < 0)
        return;
    const int slot = idx::row_slot(L, E, w.pass, w.k, w.r);
    if (w.table >= 0) {
        rows[slot] = tw[w.table];
    } else {
        double sn, cs;
        sincospi(2.0 * (double)(w.r * w.k) / (double)(1 << w.mlog2), &sn, &cs);
        rows[slot] = float2{(float)cs, (float)(-sn)};
    }
}

hipError_t launch_twiddle_rows(const void* tw, void* rows, int L, int E, int total, hipStream_t stream)
{
    if (total <= 0)
        return hipSuccess;
    return launch_kernel(k_twiddle_rows, dim3((total + 255) / 256), dim3(256), 0, stream,
                       static_cast<const float2*>(tw), static_cast<float2*>(rows), L, E, total);
}

}  // namespace mifft

namespace mifft {

// Twiddles of the real-input split: wn[k] = w_n^k = exp(-2 pi i k / n) for
// k < n/2.  Copies of the 2048-entry table for n <= 2048 (twiddles
// identical to the complex kernels'); FP64 sincospi rounded once above.
__global__ void k_twiddle_real(const float2* __restrict__ tw, float2* __restrict__ wn, int log2n)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (1 << (log2n - 1)))
        return;
    if (log2n <= 11) {
        wn[k] = tw[k << (11 - log2n)];
    } else {
        double sn, cs;
        sincospi(2.0 * (double)k / (double)(1 << log2n), &sn, &cs);
        wn[k] = float2{(float)cs, (float)(-sn)};
    }
}

hipError_t launch_twiddle_real(const void* tw, void* wn, int log2n, hipStream_t stream)
{
    const int m = 1 << (log2n - 1);
    return launch_kernel(k_twiddle_real, dim3((m + 255) / 256), dim3(256), 0, stream, static_cast<const float2*>(tw),
                       static_cast<float2*>(wn), log2n);
}

}  // namespace mifft

namespace mifft {

// The even/odd split of the real-input transforms above 2^15 (see
// real.hip for the formulas), one thread per bin pair (k, M - k),
// k = 0..M/2, so both halves of a transform are read and written in
// ascending / descending runs.
struct cf2 {
    float x, y;
};

__device__ __forceinline__ cf2 cmul2(cf2 a, cf2 b) { return cf2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }

// X_k from a = Z_k, b = Z_{M-k}, w = w_n^k.
__device__ __forceinline__ cf2 split_bin(cf2 a, cf2 b, cf2 w)
{
    const float sx = 0.5f * (a.x + b.x), sy = 0.5f * (a.y - b.y);
    const float dx = 0.5f * (a.y + b.y), dy = -0.5f * (a.x - b.x);
    return cf2{sx + w.x * dx - w.y * dy, sy + w.x * dy + w.y * dx};
}

// Z'_k from a = X_k, b = X_{M-k}, w = w_n^k.
__device__ __forceinline__ cf2 unsplit_bin(cf2 a, cf2 b, cf2 w)
{
    const float dx = a.x - b.x, dy = a.y + b.y;
    return cf2{a.x + b.x - w.x * dy + w.y * dx, a.y - b.y + w.x * dx + w.y * dy};
}

template <int DIR>
__global__ __launch_bounds__(256) void k_real_split(const cf2* __restrict__ src, cf2* __restrict__ dst,
                                                    const cf2* __restrict__ tlo, const cf2* __restrict__ thi,
                                                    int log2m, int64_t kblocks, float we, float wi)
{
    const int64_t M = int64_t(1) << log2m;
    const int64_t b = blockIdx.x / kblocks;
    const int64_t k = (blockIdx.x % kblocks) * 256 + threadIdx.x;
    if (k > M / 2)
        return;
    const int64_t kp = (M - k) & (M - 1);  // partner bin (k = 0 pairs with itself in Z)
    const cf2 w = cmul2(thi[k >> 10], tlo[k & 1023]);        // w_n^k
    const cf2 wp = cmul2(thi[(M - k) >> 10], tlo[(M - k) & 1023]);  // w_n^{M-k}
    if (DIR == 0) {
        const cf2* z = src + b * M;
        cf2* x = dst + b * (M + 1);
        const cf2 a = z[k], c = z[kp];
        const float s = k == 0 ? we : wi;
        const cf2 xk = split_bin(a, c, w);
        x[k] = cf2{xk.x * s, xk.y * s};
        if (k == 0) {
            x[M] = cf2{(a.x - a.y) * we, 0.f};  // X_M = E_0 - O_0
        } else if (k != M / 2) {
            const cf2 xm = split_bin(c, a, wp);
            x[M - k] = cf2{xm.x * wi, xm.y * wi};
        }
    } else {
        const cf2* x = src + b * (M + 1);
        cf2* z = dst + b * M;
        cf2 a = x[k], c = x[M - k];
        if (k == 0) {
            a.y = 0.f;
            c.y = 0.f;
        }
        const float s = k == 0 ? we : wi;
        const cf2 zk = unsplit_bin(a, c, w);
        z[k] = cf2{zk.x * s, zk.y * s};
        if (k != 0 && k != M / 2) {
            const cf2 zm = unsplit_bin(c, a, wp);
            z[M - k] = cf2{zm.x * wi, zm.y * wi};
        }
    }
}

hipError_t launch_real_split(int dir, const void* src, void* dst, const void* tlo, const void* thi, int log2n,
                             int64_t batch, float we, float wi, hipStream_t stream)
{
    const int log2m = log2n - 1;
    const int64_t kblocks = (((int64_t(1) << log2m) / 2 + 1) + 255) / 256;
    const dim3 grid((unsigned)(kblocks * batch));
    if (dir == 0)
        return launch_kernel(k_real_split<0>, grid, dim3(256), 0, stream, static_cast<const cf2*>(src),
                           static_cast<cf2*>(dst), static_cast<const cf2*>(tlo), static_cast<const cf2*>(thi), log2m,
                           kblocks, we, wi);
    else
        return launch_kernel(k_real_split<1>, grid, dim3(256), 0, stream, static_cast<const cf2*>(src),
                           static_cast<cf2*>(dst), static_cast<const cf2*>(tlo), static_cast<const cf2*>(thi), log2m,
                           kblocks, we, wi);
}

}  // namespace mifft
