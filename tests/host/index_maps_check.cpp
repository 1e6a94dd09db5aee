// Host build of the kernels' index maps (paper_2203_09384_amd/csrc/index_maps.hpp)
// for the CPU tests: thin extern "C" wrappers, bulk where the tests sweep
// every index.  No GPU code, no arithmetic of the transform itself.
#include <stdint.h>

#include "index_maps.hpp"
#include "nd_maps.hpp"

using namespace mifft::idx;

extern "C" {

int im_np(int L, int E) { return sched_np(L, E); }
int im_log2r(int L, int E, int p) { return sched_log2r(L, E, p); }
int im_log2ns(int L, int E, int p) { return sched_log2ns(L, E, p); }

// out[j * R + r] = destination of output r of butterfly j in pass p
void im_pass_dsts(int L, int E, int p, int* out)
{
    const int R = 1 << sched_log2r(L, E, p), nb = (1 << L) / R;
    for (int j = 0; j < nb; j++)
        for (int r = 0; r < R; r++)
            out[j * R + r] = stockham_dst(L, E, p, j, r);
}

int im_rows_offset(int L, int E, int P) { return rows_offset(L, E, P); }
int im_rows_total(int L, int E) { return rows_total(L, E); }

// out[5 i .. 5 i + 4] = (pass, r, k, mlog2, table) of row entry i, i < count
void im_row_entries(int L, int E, int count, int* out)
{
    for (int i = 0; i < count; i++) {
        const RowEntry w = twiddle_row_entry(L, E, i);
        out[5 * i] = w.pass;
        out[5 * i + 1] = w.r;
        out[5 * i + 2] = w.k;
        out[5 * i + 3] = w.mlog2;
        out[5 * i + 4] = w.table;
    }
}

int im_pad_bits(int L, int E, int P) { return pad_bits(L, E, P); }

// out[i] = storage slot of row entry i (row-major numbering)
void im_row_slots(int L, int E, int count, int* out)
{
    for (int i = 0; i < count; i++) {
        const RowEntry w = twiddle_row_entry(L, E, i);
        out[i] = w.pass < 0 ? -1 : row_slot(L, E, w.pass, w.k, w.r);
    }
}
int im_pad_index(int B, int d) { return pad_index(B, d); }
int im_region(int L, int E) { return region(L, E); }
int im_pad_is_affine(int L, int E, int P, int B) { return pad_is_affine(L, E, P, B) ? 1 : 0; }
void im_strides(int L, int E, int P, int* out)
{
    const Strides s = exchange_strides(L, E, P);
    out[0] = s.B;
    out[1] = s.DR;
    out[2] = s.DQ;
    out[3] = s.DM;
}

void im_xcd_group_tiles(int64_t n, int G, int64_t* out)
{
    for (int64_t b = 0; b < n; b++)
        out[b] = xcd_group_tile(b, G);
}

// out[q * N + n] = axis_elem(q, n), q < count, n < N = 2^L
void im_axis_elems(int64_t count, int L, int log2s, int64_t* out)
{
    for (int64_t q = 0; q < count; q++)
        for (int64_t n = 0; n < (int64_t(1) << L); n++)
            out[(q << L) + n] = axis_elem(q, n, L, log2s);
}

// column pass of the four-step split: out_in[(tile, c, n1)] and out_out[(tile, c, k1)]
void im_fourstep_cols(int64_t ntiles, int L1, int L2, int T, int64_t* out_in, int64_t* out_out)
{
    const int N1 = 1 << L1;
    for (int64_t t = 0; t < ntiles; t++)
        for (int c = 0; c < T; c++)
            for (int n = 0; n < N1; n++) {
                const int64_t i = (t * T + c) * N1 + n;
                out_in[i] = fourstep_col_in(t, c, n, L1, L2, T);
                out_out[i] = fourstep_col_out(t, c, n, L1, L2, T);
            }
}

int im_real_partner(int M, int k) { return real_partner(M, k); }

// single-pass 2D: out = fits, E, TPA, AP, WG, TPT0, TPT1, RS1, RS0, ASZ, LDS
void im_nd2_geom(int L0, int L1, int* out)
{
    const mifft::ndm::Nd2Geom g = mifft::ndm::nd2_geom(L0, L1);
    const int v[] = {mifft::ndm::nd2_fits(L0, L1) ? 1 : 0, g.E, g.TPA, g.AP, g.WG, g.TPT0, g.TPT1, g.RS1, g.RS0,
                     g.ASZ, g.LDS};
    for (int i = 0; i < 11; i++)
        out[i] = v[i];
}

// out[r N1 + k1] = the turn's LDS index of point k1 of row r
void im_nd2_turns(int L0, int L1, int* out)
{
    const mifft::ndm::Nd2Geom g = mifft::ndm::nd2_geom(L0, L1);
    for (int r = 0; r < g.N0; r++)
        for (int k = 0; k < g.N1; k++)
            out[r * g.N1 + k] = mifft::ndm::nd2_turn(r, k, g.RS0);
}

// single-pass 3D: out = fits, E, TPA, AP, WG, TPT0, TPT1, TPT2, RS2, RS1,
// RS0, A2, A1, A0, ASZ, LDS
void im_nd3_geom(int L0, int L1, int L2, int* out)
{
    const mifft::ndm::Nd3Geom g = mifft::ndm::nd3_geom(L0, L1, L2);
    const int v[] = {mifft::ndm::nd3_fits(L0, L1, L2) ? 1 : 0, g.E, g.TPA, g.AP, g.WG, g.TPT0, g.TPT1, g.TPT2, g.RS2,
                     g.RS1, g.RS0, g.A2, g.A1, g.A0, g.ASZ, g.LDS};
    for (int i = 0; i < 16; i++)
        out[i] = v[i];
}

// t21[(i0 N1 + i1) N2 + k2]: the first turn's LDS index of point k2 of row
// (i0, i1); t10[(i0 N1 + k1) N2 + k2]: the second turn's of point k1 of the
// axis-1 line (i0, k2)
void im_nd3_turns(int L0, int L1, int L2, int* t21, int* t10)
{
    const mifft::ndm::Nd3Geom g = mifft::ndm::nd3_geom(L0, L1, L2);
    for (int i0 = 0; i0 < g.N0; i0++)
        for (int j = 0; j < g.N1; j++)
            for (int k2 = 0; k2 < g.N2; k2++) {
                t21[(i0 * g.N1 + j) * g.N2 + k2] = mifft::ndm::nd3_turn21(i0, j, k2, g.N2, g.RS1);
                t10[(i0 * g.N1 + j) * g.N2 + k2] = mifft::ndm::nd3_turn10(i0, j, k2, g.N2, g.RS0);
            }
}

}  // extern "C"
