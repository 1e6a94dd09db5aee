"""CPU checks of the kernels' index maps.

The kernels take their Stockham schedules, LDS exchange layouts,
twiddle-row tables, tile-to-workgroup maps and four-step / axis / real-input
addressing from paper_2203_09384_amd/csrc/index_maps.hpp.  Here the same
header is built for the host (g++) and enumerated:

* every Stockham schedule (length 2^1..2^14, 2..16 elements per thread),
  driven by the exported destination map and twiddle-row entries, reproduces
  the DFT of Eq. (dft) -- the bookkeeping of the Cooley-Tukey split of
  Eq. (radix2) with radix R;
* every twiddle-row entry indexes the 2048-entry table inside [0, 2048), and
  exactly the rows of passes longer than 2048 points go to FP64 instead (an
  out-of-bounds index there once faulted the GPU);
* every padded LDS exchange's affine addresses equal the padded Stockham
  addresses, distinct and inside the region;
* the XCD tile grouping is a bijection that puts tiles sharing 128-byte
  lines on one XCD; axis and four-step maps touch every element exactly
  once, and the four-step maps reproduce the DFT;
* the real-input partner map pairs bins as the even/odd split needs;
* the single-pass 2D / 3D kernels' geometry and turns through LDS
  (paper_2203_09384_amd/csrc/nd_maps.hpp): every turn injective and in
  bounds, every line's exchange region inside its stride, and the dataflow
  rows -> turn -> lines (-> turn -> lines) reproducing the 2D / 3D DFT for
  every shape the kernels are built for.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2203_09384_amd", "csrc")

I32P = ctypes.POINTER(ctypes.c_int)
I64P = ctypes.POINTER(ctypes.c_int64)


@pytest.fixture(scope="module")
def im(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("im") / "libindexmaps.so")
    cmd = ["g++", "-O1", "-std=c++17", "-Wall", "-Werror", "-fPIC", "-shared", f"-I{CSRC}",
           os.path.join(HERE, "host", "index_maps_check.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return ctypes.CDLL(out)


def ip(a):
    return a.ctypes.data_as(I32P)


def lp(a):
    return a.ctypes.data_as(I64P)


def row_entries(im, L, E):
    n = im.im_rows_total(L, E)
    out = np.zeros(5 * max(n, 1), np.int32)
    im.im_row_entries(L, E, n, ip(out))
    return out[: 5 * n].reshape(n, 5)


def schedules():
    return [(L, E) for L in range(1, 15) for E in range(1, 5) if E <= L]


def stockham_emulation(im, L, E, x):
    """Run the passes of schedule (L, E) on x (sign -1) with the exported
    destination map and the twiddles named by the exported row entries."""
    N = 1 << L
    rows = row_entries(im, L, E)
    X = x.astype(np.complex128).copy()
    for p in range(im.im_np(L, E)):
        lr, lns = im.im_log2r(L, E, p), im.im_log2ns(L, E, p)
        R, NS, nb = 1 << lr, 1 << lns, N >> lr
        j = np.arange(nb)
        y = np.stack([X[j + r * nb] for r in range(R)], axis=1)  # input r of butterfly j
        if NS > 1:
            assert R == 1 << E, "twiddled passes have radix EPT"
            ent = rows[im.im_rows_offset(L, E, p) + (j & (NS - 1))[:, None] * (1 << E) + np.arange(R)[None, :]]
            assert np.all(ent[..., 0] == p) and np.all(ent[..., 1] == np.arange(R)[None, :])
            assert np.all(ent[..., 2] == (j & (NS - 1))[:, None])
            from_table = ent[..., 4] >= 0
            val = np.where(from_table, np.exp(-2j * np.pi * ent[..., 4] / 2048.0),
                           np.exp(-2j * np.pi * (ent[..., 1] * ent[..., 2]) / 2.0 ** ent[..., 3]))
            y = y * val
        Y = np.fft.fft(y, axis=1)  # the radix-R butterfly: DFT_R over r
        dst = np.zeros(nb * R, np.int32)
        im.im_pass_dsts(L, E, p, ip(dst))
        assert np.array_equal(np.sort(dst), np.arange(N)), "a pass writes every position once"
        out = np.empty(N, np.complex128)
        out[dst] = Y.reshape(-1)
        X = out
    return X


@pytest.mark.parametrize("L,E", schedules())
def test_stockham_schedule_reproduces_the_dft(im, L, E):
    x = np.random.default_rng(L * 8 + E).standard_normal((1 << L, 2)) @ np.array([1.0, 1j])
    got = stockham_emulation(im, L, E, x)
    ref = np.fft.fft(x)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("L,E", schedules())
def test_twiddle_rows_stay_inside_the_table(im, L, E):
    rows = row_entries(im, L, E)
    if len(rows) == 0:
        return
    p, r, k, mlog2, table = rows.T
    assert np.all(p >= 1) and np.all((r >= 0) & (r < (1 << E)))
    assert np.all(mlog2 == np.array([im.im_log2ns(L, E, int(q)) for q in p]) + E)
    assert np.all((k >= 0) & (k < (1 << (mlog2 - E))))
    in_table = mlog2 <= 11
    assert np.all(table[~in_table] == -1), "rows of passes above 2048 points are evaluated in FP64"
    t = table[in_table]
    assert np.all((t >= 0) & (t < 2048))
    assert np.all(t * (1 << mlog2[in_table]) == 2048 * (r[in_table] * k[in_table]))


@pytest.mark.parametrize("L,E", schedules())
def test_row_storage_is_a_permutation(im, L, E):
    """Row entries are stored row-major up to 4096 points and entry-major
    within each pass from 8192 up (the single-pass kernels of those lengths
    read every pass's rows once per transform, consecutive lanes taking
    consecutive rows): either way a permutation of the table that keeps
    each pass inside its own region."""
    n = im.im_rows_total(L, E)
    if n == 0:
        return
    slots = np.zeros(n, np.int32)
    im.im_row_slots(L, E, n, ip(slots))
    assert np.array_equal(np.sort(slots), np.arange(n))
    rows = row_entries(im, L, E)
    p, r, k = rows[:, 0], rows[:, 1], rows[:, 2]
    off = np.array([im.im_rows_offset(L, E, int(q)) for q in p])
    ns = 1 << np.array([im.im_log2ns(L, E, int(q)) for q in p])
    if L >= 13:
        assert np.array_equal(slots, off + r * ns + k)
    else:
        assert np.array_equal(slots, np.arange(n))


@pytest.mark.parametrize("L,E", [(L, E) for L in range(2, 15) for E in range(2, 5) if E < L])
def test_padded_exchanges_are_affine_distinct_and_in_bounds(im, L, E):
    N, EPT = 1 << L, 1 << E
    TPT = N // EPT
    reg = im.im_region(L, E)
    t = np.arange(TPT)
    for P in range(im.im_np(L, E) - 1):
        st = np.zeros(4, np.int32)
        im.im_strides(L, E, P, ip(st))
        B, DR, DQ, DM = (int(v) for v in st)
        assert B == im.im_pad_bits(L, E, P) and im.im_pad_is_affine(L, E, P, B)
        pad = np.vectorize(lambda d: im.im_pad_index(B, int(d)))
        lr = im.im_log2r(L, E, P)
        R, Q = 1 << lr, EPT >> lr
        dst = np.zeros(N, np.int32)
        im.im_pass_dsts(L, E, P, ip(dst))
        dst = dst.reshape(N // R, R)
        d0 = pad(dst[t, 0])
        wr_affine = d0[:, None, None] + DQ * np.arange(Q)[None, :, None] + DR * np.arange(R)[None, None, :]
        wr_exact = pad(dst[t[:, None, None] + TPT * np.arange(Q)[None, :, None], np.arange(R)[None, None, :]])
        assert np.array_equal(wr_affine, wr_exact)
        assert len(np.unique(wr_exact)) == N and wr_exact.max() < reg
        rd_affine = pad(t)[:, None] + DM * np.arange(EPT)[None, :]
        rd_exact = pad(t[:, None] + TPT * np.arange(EPT)[None, :])
        assert np.array_equal(rd_affine, rd_exact)
        # the reads of pass P + 1 see exactly the slots written by pass P
        assert np.array_equal(np.sort(rd_exact.reshape(-1)), np.sort(wr_exact.reshape(-1)))


@pytest.mark.parametrize("G", [2, 4])
def test_xcd_grouping(im, G):
    n = 8 * G * 7
    tiles = np.zeros(n, np.int64)
    im.im_xcd_group_tiles(n, G, lp(tiles))
    assert np.array_equal(np.sort(tiles), np.arange(n))
    b = np.arange(n)
    # the G tiles G i .. G i + G - 1 of a chunk run on blocks of one XCD (b mod 8)
    xcd_of_tile = np.empty(n, np.int64)
    xcd_of_tile[tiles] = b % 8
    assert np.all(xcd_of_tile.reshape(-1, G) == xcd_of_tile.reshape(-1, G)[:, :1])


@pytest.mark.parametrize("L,log2s,arrays", [(1, 0, 3), (3, 4, 2), (5, 0, 4), (4, 7, 2), (11, 1, 2), (7, 6, 1),
                                             (2, 11, 1)])
def test_axis_map_covers_every_element_once(im, L, log2s, arrays):
    total = arrays << (L + log2s)
    count = total >> L
    out = np.zeros(total, np.int64)
    im.im_axis_elems(count, L, log2s, lp(out))
    assert np.array_equal(np.sort(out), np.arange(total))
    # point n of a transform is 2^log2s elements after point n - 1
    a = out.reshape(count, 1 << L)
    if L > 0:
        assert np.all(np.diff(a, axis=1) == (1 << log2s))


def col_tile(L1):
    return 8 if L1 >= 10 else 16


@pytest.mark.parametrize("L", [12, 13, 15, 16, 20])
def test_fourstep_maps_reproduce_the_dft(im, L):
    """The four-step split N = N1 N2 with the exported column-pass maps
    (inputs, outputs Y[k1 + N1 n2]) and the axis map for the row pass
    (stride N1), against numpy's FFT."""
    L1, L2 = (L + 1) // 2, L // 2
    N1, N2, N = 1 << L1, 1 << L2, 1 << L
    T = col_tile(L1)
    batch = 2
    ntiles = batch * N2 // T
    fin = np.zeros(ntiles * T * N1, np.int64)
    fout = np.zeros_like(fin)
    im.im_fourstep_cols(ntiles, L1, L2, T, lp(fin), lp(fout))
    assert np.array_equal(np.sort(fin), np.arange(batch * N))
    assert np.array_equal(np.sort(fout), np.arange(batch * N))
    x = np.random.default_rng(L).standard_normal((batch * N, 2)) @ np.array([1.0, 1j])
    cols = x[fin].reshape(ntiles, T, N1)                     # column (tile, c), points n1
    n2 = (np.arange(ntiles) % (N2 // T))[:, None] * T + np.arange(T)[None, :]
    k1 = np.arange(N1)
    Ycol = np.fft.fft(cols, axis=2) * np.exp(-2j * np.pi * n2[:, :, None] * k1[None, None, :] / N)
    Y = np.empty(batch * N, np.complex128)
    Y[fout] = Ycol.reshape(-1)
    # row pass: transforms of N2 points at stride N1, batch * N1 of them, in place
    ax = np.zeros(batch * N, np.int64)
    im.im_axis_elems(batch * N1, L2, L1, lp(ax))
    ax = ax.reshape(batch * N1, N2)
    Xf = np.empty_like(Y)
    Xf[ax] = np.fft.fft(Y[ax], axis=1)
    ref = np.fft.fft(x.reshape(batch, N), axis=1).reshape(-1)
    assert np.linalg.norm(Xf - ref) <= 1e-11 * np.linalg.norm(ref)


@pytest.mark.parametrize("M", [1, 2, 4, 8, 1024, 16384])
def test_real_partner_map_gives_the_split(im, M):
    part = np.array([im.im_real_partner(M, k) for k in range(M)])
    assert part[0] == 0 and np.array_equal(part[part], np.arange(M))
    assert np.array_equal(part[1:], M - np.arange(1, M))
    # the even/odd split of Eq. (radix2) on Z = DFT_M(x_even + i x_odd)
    x = np.random.default_rng(M).standard_normal(2 * M)
    Z = np.fft.fft(x[0::2] + 1j * x[1::2])
    Zp = np.conj(Z[part])
    k = np.arange(M)
    X = 0.5 * (Z + Zp) + np.exp(-2j * np.pi * k / (2 * M)) * (Z - Zp) / 2j
    assert np.allclose(X, np.fft.rfft(x)[:M], rtol=0, atol=1e-10 * np.abs(x).sum())


# ---------------------------------------------------------------- single-pass 2D / 3D
def nd2_shapes():
    return [(a, b) for a in range(1, 14) for b in range(1, 14) if a + b <= 14]


def nd3_shapes():
    return [(a, b, c) for a in range(2, 11) for b in range(2, 11) for c in range(2, 11) if a + b + c <= 14]


def test_single_pass_shape_counts(im):
    """The shapes the kernels exist for (every axis from 2 (2D) or 4 (3D)
    points, at most 16384 points, 1024 threads and 160 KiB of LDS; rows
    inside one wavefront)."""
    g2 = np.zeros(11, np.int32)
    g3 = np.zeros(16, np.int32)
    n2 = sum(im.im_nd2_geom(a, b, ip(g2)) or int(g2[0]) for a, b in nd2_shapes())
    n3 = sum(im.im_nd3_geom(a, b, c, ip(g3)) or int(g3[0]) for a, b, c in nd3_shapes())
    assert n3 == 100 and n2 > 50
    assert not im.im_nd3_geom(4, 5, 5, ip(g3)) and g3[0] == 0  # 16 x 32 x 32: 196 KiB of LDS


@pytest.mark.parametrize("L0,L1", nd2_shapes())
def test_single_pass_2d_maps_reproduce_the_dft(im, L0, L1):
    """Rows into their regions, the turn, columns read at stride RS0 and
    stored X[k0][c]: the dataflow of the single-pass 2D kernel with each
    line's transform taken as a DFT (the Stockham passes are checked
    above), against the 2D DFT."""
    g = np.zeros(11, np.int32)
    im.im_nd2_geom(L0, L1, ip(g))
    fits, E, TPA, AP, WG, TPT0, TPT1, RS1, RS0, ASZ, LDS = (int(v) for v in g)
    if not fits:
        return
    N0, N1 = 1 << L0, 1 << L1
    assert TPA == N0 * N1 >> E and TPT0 == N0 >> E and TPT1 == N1 >> E and TPT1 <= 64
    assert WG == AP * TPA and LDS == AP * ASZ * 8 <= 160 * 1024
    # rows: region r at r RS1 holds the row's exchanges; columns: line c at c RS0
    assert RS1 >= im.im_region(L1, E) and N0 * RS1 <= ASZ
    assert RS0 % 2 == 1 and RS0 >= im.im_region(L0, E) and (N1 - 1) * RS0 + im.im_region(L0, E) <= ASZ
    turn = np.zeros(N0 * N1, np.int32)
    im.im_nd2_turns(L0, L1, ip(turn))
    assert len(np.unique(turn)) == N0 * N1 and turn.min() >= 0 and turn.max() < ASZ
    x = np.random.default_rng(L0 * 16 + L1).standard_normal((N0, N1, 2)) @ np.array([1.0, 1j])
    rows = np.fft.fft(x, axis=1)
    lds = np.full(ASZ, np.nan + 0j)
    lds[turn] = rows.reshape(-1)
    cols = lds[np.arange(N1)[:, None] * RS0 + np.arange(N0)[None, :]]  # line c, point n
    assert not np.isnan(cols).any()
    out = np.fft.fft(cols, axis=1).T  # out[k0][c]
    ref = np.fft.fft2(x)
    assert np.linalg.norm(out - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("L0,L1,L2", nd3_shapes())
def test_single_pass_3d_maps_reproduce_the_dft(im, L0, L1, L2):
    """Axis-2 rows, the turn to the axis-1 lines (i0, k2) at stride RS1, the
    turn to the axis-0 lines (k1, k2) at stride RS0, stored X[k0][k1][k2]:
    the dataflow of the single-pass 3D kernel with each line's transform
    taken as a DFT, against the 3D DFT."""
    g = np.zeros(16, np.int32)
    im.im_nd3_geom(L0, L1, L2, ip(g))
    fits, E, TPA, AP, WG, TPT0, TPT1, TPT2, RS2, RS1, RS0, A2, A1, A0, ASZ, LDS = (int(v) for v in g)
    if not fits:
        return
    N0, N1, N2 = 1 << L0, 1 << L1, 1 << L2
    assert E == min(L0, L1, L2, 4) and TPA == (N0 * N1 * N2) >> E and TPT2 <= 64
    assert (TPT0, TPT1, TPT2) == (N0 >> E, N1 >> E, N2 >> E)
    assert ASZ == max(A2, A1, A0) and LDS == AP * ASZ * 8 <= 160 * 1024 and WG == AP * TPA
    assert RS2 >= im.im_region(L2, E) and A2 == N0 * N1 * RS2
    for L, RS, lines, A in ((L1, RS1, N0 * N2, A1), (L0, RS0, N1 * N2, A0)):
        assert RS % 2 == 1 and RS >= im.im_region(L, E) and (lines - 1) * RS + im.im_region(L, E) <= A
    t21 = np.zeros(N0 * N1 * N2, np.int32)
    t10 = np.zeros(N0 * N1 * N2, np.int32)
    im.im_nd3_turns(L0, L1, L2, ip(t21), ip(t10))
    for t in (t21, t10):
        assert len(np.unique(t)) == t.size and t.min() >= 0 and t.max() < ASZ
    x = np.random.default_rng(L0 * 256 + L1 * 16 + L2).standard_normal((N0, N1, N2, 2)) @ np.array([1.0, 1j])
    rows = np.fft.fft(x, axis=2)  # rows[i0, i1, k2]
    lds = np.full(ASZ, np.nan + 0j)
    lds[t21] = rows.reshape(-1)
    l1 = lds[np.arange(N0 * N2)[:, None] * RS1 + np.arange(N1)[None, :]]  # line (i0, k2), point i1
    assert not np.isnan(l1).any()
    y1 = np.fft.fft(l1, axis=1).reshape(N0, N2, N1).transpose(0, 2, 1)  # y1[i0, k1, k2]
    lds = np.full(ASZ, np.nan + 0j)
    lds[t10] = y1.reshape(-1)
    l0 = lds[np.arange(N1 * N2)[:, None] * RS0 + np.arange(N0)[None, :]]  # line (k1, k2), point i0
    assert not np.isnan(l0).any()
    out = np.fft.fft(l0, axis=1).T.reshape(N0, N1, N2)  # stored at k0 N1 N2 + c
    ref = np.fft.fftn(x)
    assert np.linalg.norm(out - ref) <= 1e-12 * np.linalg.norm(ref)
