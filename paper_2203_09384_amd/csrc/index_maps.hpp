// Index maps of the kernels as constexpr functions that compile for the
// host and the device.  The kernels compute their schedules, LDS layouts,
// twiddle-row tables and tile assignments with these, and a host-only test
// build enumerates the same functions: every address in bounds, every
// permutation a permutation, and the Stockham bookkeeping of every
// (length, elements per thread) reproducing the DFT.
#pragma once
#include <stdint.h>

#if defined(__HIP__)
#define MIFFT_HD __host__ __device__
#else
#define MIFFT_HD
#endif

namespace mifft {
namespace idx {

// ---------------------------------------------------------------- Stockham schedule
// log2 N = a log2 EPT + rem: a radix-2^rem pass first (NS = 1), then passes
// of radix EPT.  NS = product of the radices of the passes before p.
MIFFT_HD constexpr int sched_np(int L, int E) { return L / E + (L % E ? 1 : 0); }
MIFFT_HD constexpr int sched_log2r(int L, int E, int p) { return (L % E && p == 0) ? L % E : E; }
MIFFT_HD constexpr int sched_log2ns(int L, int E, int p)
{
    return p == 0 ? 0 : (L % E ? L % E + (p - 1) * E : p * E);
}

// Pass p (radix R = 2^LR, NS = 2^LNS) writes output r of butterfly j
// (k = j mod NS) to (j - k) R + k + r NS: the self-sorting form of the
// Cooley-Tukey step of Eq. (radix2) with radix R.
MIFFT_HD constexpr int stockham_dst(int L, int E, int p, int j, int r)
{
    const int lr = sched_log2r(L, E, p), lns = sched_log2ns(L, E, p);
    return ((j >> lns) << (lns + lr)) + (j & ((1 << lns) - 1)) + (r << lns);
}

// ---------------------------------------------------------------- twiddle rows
// For each pass with NS > 1 (radix EPT), NS rows of EPT entries: row k holds
// w_M^{r k}, M = NS EPT, r < EPT.  Rows of pass p start at rows_offset(p).
MIFFT_HD constexpr int rows_offset(int L, int E, int P)
{
    int off = 0;
    for (int p = 0; p < P; p++)
        if (sched_log2ns(L, E, p) > 0)
            off += (1 << sched_log2ns(L, E, p)) << E;
    return off;
}
MIFFT_HD constexpr int rows_total(int L, int E) { return rows_offset(L, E, sched_np(L, E)); }

// What entry i of the rows of schedule (L, E) holds: w_{2^mlog2}^{rk}.  When
// M <= 2048 it is the copy tw[table] of the 2048-entry table
// tw[m] = exp(-2 pi i m / 2048) (table = rk 2048 / M, always in [0, 2048));
// longer M is not resolved by the table (table = -1: evaluate in FP64).
struct RowEntry {
    int pass, r, k, mlog2, table;
};
MIFFT_HD constexpr RowEntry twiddle_row_entry(int L, int E, int i)
{
    int off = 0;
    for (int p = 0; p < sched_np(L, E); p++) {
        const int lns = sched_log2ns(L, E, p);
        if (lns == 0)
            continue;
        const int size = (1 << lns) << E;
        if (i < off + size) {
            const int k = (i - off) >> E, r = (i - off) & ((1 << E) - 1);
            const int shift = 11 - lns - E;
            return RowEntry{p, r, k, lns + E, shift >= 0 ? (r * k) << shift : -1};
        }
        off += size;
    }
    return RowEntry{-1, 0, 0, 0, -1};
}

// Where entry r of row k of pass P is stored.  Row-major (rows_offset(P) +
// k EPT + r) for transforms of up to 4096 points, whose kernels keep the
// rows or share them across transforms; entry-major within each pass
// (rows_offset(P) + r NS + k) from 8192 points up, whose kernels read every
// pass's rows once per transform: there a lane's row-major row puts lanes a
// whole row (EPT values) apart, entry-major puts consecutive k, i.e.
// consecutive lanes, at consecutive addresses.
MIFFT_HD constexpr bool rows_entry_major(int L) { return L >= 13; }
MIFFT_HD constexpr int row_slot(int L, int E, int P, int k, int r)
{
    return rows_entry_major(L) ? rows_offset(L, E, P) + r * (1 << sched_log2ns(L, E, P)) + k
                               : rows_offset(L, E, P) + (k << E) + r;
}

// ---------------------------------------------------------------- LDS exchanges
// pad(d) = d + (d >> B): one spare slot every 2^B elements, B per exchange
// (exchange P follows pass P) chosen so the writes of pass P and the reads
// of pass P + 1 stay affine in their compile-time indices and the modelled
// conflicts on the 64 LDS banks are lowest.  B = 0: no padding.
MIFFT_HD constexpr int pad_bits(int L, int E, int P)
{
    if (E == 4) {
        if (L == 5) return 1;
        if (L == 6) return 2;
        if (L == 7) return 3;
        if (L == 8) return 4;
        if (L == 9) return 5;
        if (L == 10) return P == 0 ? 5 : 6;
        if (L == 11) return P == 0 ? 5 : 3;
        if (L == 12) return P == 0 ? 5 : 4;
        if (L == 13) return 5;
        if (L == 14) return P == 1 ? 6 : 5;
    } else if (E == 3) {
        if (L == 4) return 1;
        if (L == 5) return 2;
        if (L == 6) return 3;
        if (L == 7) return P == 0 ? 1 : 4;
        if (L == 8) return P == 0 ? 5 : 2;
        if (L == 9) return P == 0 ? 5 : 3;
        if (L == 10) return P == 2 ? 7 : 5;
        if (L == 11) return P == 1 ? 2 : 5;
        if (L == 12) return P == 1 ? 3 : 5;
        if (L == 13) return P == 2 ? 7 : 5;
        if (L == 14) return P == 1 ? 2 : 5;
    } else if (E == 2) {
        if (L == 3) return 1;
        if (L == 4) return 2;
        if (L == 5) return 1;
        if (L == 6) return 2;
        if (L == 7) return P == 2 ? 1 : 5;
        if (L == 8) return P == 1 ? 2 : (P == 2 ? 6 : 5);
        if (L == 9) return P == 2 ? 1 : 5;
        if (L == 10) return P == 1 ? 2 : (P == 2 ? 6 : 5);
        if (L == 11) return P == 2 ? 1 : 5;
    }
    return 0;
}

MIFFT_HD constexpr int pad_index(int B, int d) { return B == 0 ? d : d + (d >> B); }

// LDS elements of one transform's region: N, or more where an exchange pads.
MIFFT_HD constexpr int region(int L, int E)
{
    int m = 1 << L;
    for (int p = 0; p + 1 < sched_np(L, E); p++) {
        const int B = pad_bits(L, E, p);
        const int r = B == 0 ? (1 << L) : (1 << L) + ((1 << L) >> B);
        m = r > m ? r : m;
    }
    return m;
}

// The exchange after pass P, thread t of the transform's TPT = N / EPT
// threads, Q = EPT / R butterflies per thread: writes go to
// pad(d0) + q DQ + r DR with d0 = stockham_dst(t, 0), reads of pass P + 1
// come from pad(t) + m DM.  These strides equal the padded Stockham
// addresses exactly when the padding keeps the fields of r (writes) and m
// (reads) on one side of bit B.
struct Strides {
    int B, DR, DQ, DM;
};
MIFFT_HD constexpr Strides exchange_strides(int L, int E, int P)
{
    const int lr = sched_log2r(L, E, P), lns = sched_log2ns(L, E, P);
    const int NS = 1 << lns, R = 1 << lr, TPT = (1 << L) >> E;
    const int B = pad_bits(L, E, P);
    const int DR = B == 0 ? NS : (lns >= B ? NS + (NS >> B) : NS);
    const int DQ = B == 0 ? TPT * R : (TPT * R + ((TPT * R) >> B));
    const int DM = B == 0 ? TPT : (TPT + (TPT >> B));
    return Strides{B, DR, DQ, DM};
}

MIFFT_HD constexpr bool pad_is_affine(int L, int E, int P, int B)
{
    if (B == 0 || B >= L)
        return true;
    const int lr = sched_log2r(L, E, P), lns = sched_log2ns(L, E, P);
    const int lt = L - E;
    bool w = (lns + lr <= B) || (lns >= B);
    if (E > lr)
        w = w && (lt + lr >= B);
    return w && (lt >= B);
}

// ---------------------------------------------------------------- tiles
// Workgroups are dealt round-robin over the 8 XCDs (block b on XCD b mod 8),
// each with its own L2.  When G tiles share 128-byte lines, block b of a
// chunk of 8 G blocks takes tile G (b mod 8) + (b / 8 mod G): the G tiles of
// a line go to blocks b, b + 8, ..., i.e. one XCD.  A bijection on every
// chunk.
MIFFT_HD constexpr int64_t xcd_group_tile(int64_t b, int G)
{
    return (b & ~int64_t(8 * G - 1)) + G * (b & 7) + ((b >> 3) & (G - 1));
}

// Element n of transform q of an axis of length 2^L and stride 2^log2s:
// transforms adjacent in memory are consecutive q, the array of
// 2^(L + log2s) elements repeats.
MIFFT_HD constexpr int64_t axis_elem(int64_t q, int64_t n, int L, int log2s)
{
    return ((q >> log2s) << (L + log2s)) + (n << log2s) + (q & ((int64_t(1) << log2s) - 1));
}

// Four-step split N = N1 N2 (N1 = 2^L1, N2 = 2^L2), column pass: tile
// `tile` of T columns is columns n2 = nb T + c (c < T) of transform
// b = tile / (N2 / T).  Point n1 of column c is input element n1 N2 + n2;
// output k1 of the column goes to Y[k1 + N1 n2], so a tile's outputs are
// one contiguous block.
MIFFT_HD constexpr int64_t fourstep_col_in(int64_t tile, int c, int n1, int L1, int L2, int T)
{
    const int64_t per = (int64_t(1) << L2) / T, b = tile / per, nb = tile % per;
    return (b << (L1 + L2)) + nb * T + ((int64_t)n1 << L2) + c;
}
MIFFT_HD constexpr int64_t fourstep_col_out(int64_t tile, int c, int k1, int L1, int L2, int T)
{
    const int64_t per = (int64_t(1) << L2) / T, b = tile / per, nb = tile % per;
    return (b << (L1 + L2)) + ((nb * T + c) << L1) + k1;
}

// ---------------------------------------------------------------- real input
// Bin paired with bin k of a length-M complex transform in the even/odd
// split: M - k, with bin 0 paired with itself (Z_M = Z_0).
MIFFT_HD constexpr int real_partner(int M, int k) { return (M - k) & (M - 1); }

}  // namespace idx
}  // namespace mifft
