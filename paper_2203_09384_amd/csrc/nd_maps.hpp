// Geometry and LDS index maps of the single-pass 2D and 3D kernels as
// constexpr functions that compile for the host and the device.  The
// kernels take their points per thread, arrays per workgroup, LDS strides
// and sizes and their transposes ("turns") through LDS from here, and a
// host-only test build enumerates every registered shape: turns are
// injective and in bounds, lines and rows stay inside their own regions,
// and the dataflow rows -> turn -> lines reproduces the multidimensional
// DFT (its kernel is a product over the axes, so the axes can be taken one
// after another).
#pragma once
#include "index_maps.hpp"

namespace mifft {
namespace ndm {

// log2 of the points each thread holds: the smallest axis, at most 16 points
MIFFT_HD constexpr int nd2_e(int L0, int L1)
{
    const int m = L0 < L1 ? L0 : L1;
    return m < 4 ? m : 4;
}

MIFFT_HD constexpr int nd3_e(int L0, int L1, int L2)
{
    int m = L0 < L1 ? L0 : L1;
    m = m < L2 ? m : L2;
    return m < 4 ? m : 4;
}

// Stride of a turned layout: the line's Stockham exchange region, rounded
// up to an odd number of complex values so that lanes reading consecutive
// lines spread over the 64 banks.
MIFFT_HD constexpr int line_stride(int L, int E)
{
    const int r = idx::region(L, E);
    return (r & 1) ? r : r + 1;
}

// arrays per workgroup: at least 256 threads
MIFFT_HD constexpr int arrays_per_wg(int tpa) { return tpa >= 256 ? 1 : 256 / tpa; }

// ---------------------------------------------------------------- 2D
// rows (axis 1) in regions of RS1, then columns (axis 0) at stride RS0
struct Nd2Geom {
    int E, N0, N1, TPA, AP, WG, TPT0, TPT1, RS1, RS0, ASZ, LDS;
};

MIFFT_HD constexpr Nd2Geom nd2_geom(int L0, int L1)
{
    const int E = nd2_e(L0, L1), N0 = 1 << L0, N1 = 1 << L1, TPA = (N0 * N1) >> E, AP = arrays_per_wg(TPA);
    const int RS1 = idx::region(L1, E), RS0 = line_stride(L0, E);
    const int ASZ = N0 * RS1 > N1 * RS0 ? N0 * RS1 : N1 * RS0;
    return Nd2Geom{E, N0, N1, TPA, AP, AP * TPA, N0 >> E, N1 >> E, RS1, RS0, ASZ, AP * ASZ * 8};
}

// the kernel exists for: at most 16384 points, at most 1024 threads, a row
// inside one wavefront, the arrays inside 160 KiB of LDS
MIFFT_HD constexpr bool nd2_fits(int L0, int L1)
{
    if (L0 < 1 || L1 < 1 || L0 + L1 > 14)
        return false;
    const Nd2Geom g = nd2_geom(L0, L1);
    return g.TPA <= 1024 && g.TPT1 <= 64 && g.LDS <= 160 * 1024;
}

// turn: point k1 of row r's result goes to column k1's line, position r
MIFFT_HD constexpr int nd2_turn(int r, int k1, int RS0) { return k1 * RS0 + r; }

// ---------------------------------------------------------------- 3D
// rows (axis 2, r = i0 N1 + i1) in regions of RS2, then axis-1 lines
// (i0, i2) at stride RS1, then axis-0 lines (i1, i2) at stride RS0
struct Nd3Geom {
    int E, N0, N1, N2, TPA, AP, WG, TPT0, TPT1, TPT2, RS2, RS1, RS0, A2, A1, A0, ASZ, LDS;
};

MIFFT_HD constexpr Nd3Geom nd3_geom(int L0, int L1, int L2)
{
    const int E = nd3_e(L0, L1, L2), N0 = 1 << L0, N1 = 1 << L1, N2 = 1 << L2;
    const int TPA = (N0 * N1 * N2) >> E, AP = arrays_per_wg(TPA);
    const int RS2 = idx::region(L2, E), RS1 = line_stride(L1, E), RS0 = line_stride(L0, E);
    const int A2 = N0 * N1 * RS2, A1 = N0 * N2 * RS1, A0 = N1 * N2 * RS0;
    const int ASZ = A2 > A1 ? (A2 > A0 ? A2 : A0) : (A1 > A0 ? A1 : A0);
    return Nd3Geom{E,   N0,  N1,  N2, TPA, AP, AP * TPA, N0 >> E, N1 >> E, N2 >> E, RS2, RS1, RS0,
                   A2, A1, A0, ASZ, AP * ASZ * 8};
}

// the kernel exists for: every axis at least 4, at most 16384 points, at
// most 1024 threads, a row inside one wavefront, the arrays inside 160 KiB
MIFFT_HD constexpr bool nd3_fits(int L0, int L1, int L2)
{
    if (L0 < 2 || L1 < 2 || L2 < 2 || L0 + L1 + L2 > 14)
        return false;
    const Nd3Geom g = nd3_geom(L0, L1, L2);
    return g.TPA <= 1024 && g.TPT2 <= 64 && g.LDS <= 160 * 1024;
}

// first turn: point k2 of row (i0, i1) goes to the axis-1 line (i0, k2),
// position i1
MIFFT_HD constexpr int nd3_turn21(int i0, int i1, int k2, int N2, int RS1) { return (i0 * N2 + k2) * RS1 + i1; }

// second turn: point k1 of the axis-1 line (i0, k2) goes to the axis-0
// line (k1, k2), position i0
MIFFT_HD constexpr int nd3_turn10(int i0, int k1, int k2, int N2, int RS0) { return (k1 * N2 + k2) * RS0 + i0; }

}  // namespace ndm
}  // namespace mifft
