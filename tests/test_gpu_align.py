"""Buffers aligned only to their element, against the FP64 oracle.

Offset views of contiguous tensors (x.view(-1)[1:1 + n*b] of a complex64
buffer is 8-byte aligned; of float32 reals or 16-bit pairs, 4-byte
aligned) are valid inputs and outputs: every plan kind must accept them
and give the same result as on freshly allocated tensors.  Pointers below
element alignment are refused with FFT_EALIGN before any launch.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2203_09384_amd import api, native, synth
from gpu_util import need_gpu, per_transform_relerr

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def offset_view(count, dtype, shape, off=1):
    """A contiguous view starting `off` elements into a fresh buffer."""
    buf = torch.empty(count + off + 1, dtype=dtype, device="cuda")
    return buf[off:off + count].view(shape)


def misalign(t, elems):
    """Offset copy of t: same values, data pointer `elems` elements past a
    fresh allocation (an allocation is 256-byte aligned)."""
    v = offset_view(t.numel(), t.dtype, t.shape, elems)
    v.copy_(t)
    return v


# (n, batch): staged one-per-thread (2, 16), staged shared (64), persistent
# (1024, 2048), single pass above 2048 (4096), four-step (2^16)
C32_CASES = [(2, 4097), (16, 1031), (64, 777), (1024, 67), (2048, 301), (4096, 9), (1 << 16, 3)]


@pytest.mark.parametrize("n,batch", C32_CASES)
@pytest.mark.parametrize("sign", [-1, 1])
def test_c32_offset_views(n, batch, sign):
    x = synth.uniform_complex(31, (batch, n), key=(n,))
    xv = misalign(torch.from_numpy(x).cuda(), 1)
    out = offset_view(n * batch, torch.complex64, (batch, n), 3)
    assert xv.data_ptr() % 16 == 8 and out.data_ptr() % 16 == 8
    p = api.Plan(n, batch, sign)
    print(f"[case] align c32 n={n} batch={batch} sign={sign} {p.describe()}", flush=True)
    p.execute(xv, out)
    ref = oracle.forward(x.astype(np.complex128)) if sign < 0 else oracle.inverse(x.astype(np.complex128))
    assert per_transform_relerr(out.cpu().numpy(), ref) <= TOL
    # identical to the aligned execute, bit for bit
    assert torch.equal(out, p.execute(torch.from_numpy(x).cuda()))
    # the adjoint too
    g = p.adjoint(xv)
    assert torch.equal(g, p.adjoint(torch.from_numpy(x).cuda()))


def test_ragged_and_nd_offset_views():
    lengths = synth.ragged_lengths(33, 300, 1, 11)
    off = synth.offsets_from_lengths(lengths)
    x = synth.uniform_complex(33, (int(off[-1]),), key=(1,))
    rp = api.RaggedPlan(off, -1)
    print(f"[case] align ragged {rp.describe()['tiles']} tiles", flush=True)
    y = offset_view(int(off[-1]), torch.complex64, (int(off[-1]),), 1)
    rp.execute(misalign(torch.from_numpy(x).cuda(), 1), y)
    ref = oracle.fft_ragged(x.astype(np.complex128), off, -1)
    assert torch.equal(y, rp.execute(torch.from_numpy(x).cuda()))
    yc = y.cpu().numpy()
    worst = max(np.linalg.norm(yc[a:b] - ref[a:b]) / np.linalg.norm(ref[a:b]) for a, b in zip(off[:-1], off[1:]))
    assert worst <= TOL
    for shape, batch in (((32, 32), 5), ((64, 2048), 2), ((8, 16, 32), 3)):
        x2 = synth.uniform_complex(34, (batch,) + shape)
        p = api.PlanND(shape, batch, -1)
        print(f"[case] align nd {shape} batch={batch}", flush=True)
        y2 = offset_view(x2.size, torch.complex64, (batch,) + shape, 1)
        p.execute(misalign(torch.from_numpy(x2).cuda(), 1), y2)
        ref2 = oracle.fftn(x2.astype(np.complex128), len(shape))
        assert per_transform_relerr(y2.cpu().numpy().reshape(batch, -1), ref2.reshape(batch, -1)) <= TOL


@pytest.mark.parametrize("n,batch", [(2, 1001), (64, 257), (2048, 33), (1 << 16, 3)])
def test_real_offset_views(n, batch):
    """Reals 4-byte aligned (one float past an allocation), bins 8-byte
    aligned; R2C, C2R and both adjoints against the aligned executes."""
    xr = synth.uniform_real(35, (batch, n), key=(n,))
    xa = torch.from_numpy(xr).cuda()
    xv = misalign(xa, 1)
    assert xv.data_ptr() % 8 == 4
    fwd = api.Plan(n, batch, -1, dtype="r32")
    inv = api.Plan(n, batch, +1, dtype="r32")
    print(f"[case] align r32 n={n} batch={batch}", flush=True)
    bins = offset_view(batch * (n // 2 + 1), torch.complex64, (batch, n // 2 + 1), 1)
    fwd.execute(xv, bins)
    ref = oracle.rfft(xr.astype(np.float64))
    assert per_transform_relerr(bins.cpu().numpy(), ref) <= TOL
    assert torch.equal(bins, fwd.execute(xa))
    back = offset_view(batch * n, torch.float32, (batch, n), 3)
    assert back.data_ptr() % 8 == 4
    inv.execute(bins, back)
    assert torch.equal(back, inv.execute(bins.clone()))
    assert float((back - xa).abs().max()) <= 1e-5
    # adjoints write the other side: reals at 4-byte alignment again
    adj = offset_view(batch * n, torch.float32, (batch, n), 1)
    fwd.adjoint(bins, adj)
    assert torch.equal(adj, fwd.adjoint(bins.clone()))
    adj2 = offset_view(batch * (n // 2 + 1), torch.complex64, (batch, n // 2 + 1), 1)
    inv.adjoint(xv, adj2)
    assert torch.equal(adj2, inv.adjoint(xa))


@pytest.mark.parametrize("n,batch", [(2, 3001), (64, 301), (2048, 65)])
@pytest.mark.parametrize("dtype", ["c16", "cbf16"])
def test_half_offset_views(n, batch, dtype):
    """16-bit (re, im) pairs at 4-byte alignment (one pair past an
    allocation): the same stored output and exponents as aligned buffers."""
    tdt = torch.float16 if dtype == "c16" else torch.bfloat16
    x = synth.uniform_complex(36, (batch, n), key=(n,), dtype=np.complex128)
    xa = torch.from_numpy(np.stack([x.real, x.imag], -1).astype(np.float32)).to(tdt).cuda()
    buf = torch.empty(2 * (batch * n + 2), dtype=tdt, device="cuda")
    xv = buf[2:2 + 2 * batch * n].view(batch, n, 2)
    xv.copy_(xa)
    assert xv.data_ptr() % 16 == 4
    obuf = torch.empty_like(buf)
    yv = obuf[2:2 + 2 * batch * n].view(batch, n, 2)
    p = api.Plan(n, batch, -1, dtype=dtype)
    print(f"[case] align {dtype} n={n} batch={batch}", flush=True)
    _, ev = p.execute_scaled(xv, out=yv)
    ya, ea = p.execute_scaled(xa)
    assert torch.equal(yv, ya) and torch.equal(ev, ea)


def test_fused_loss_offset_views():
    n, batch = 2048, 37
    x = synth.uniform_complex(37, (batch, n))
    w = synth.uniform_weights(37, (batch, n), key=(1,))
    p = api.Plan(n, batch, -1)
    xv = misalign(torch.from_numpy(x).cuda(), 1)
    wv = misalign(torch.from_numpy(w).cuda(), 1)
    gv = offset_view(n * batch, torch.complex64, (batch, n), 1)
    print("[case] align fused loss", flush=True)
    loss, _ = p.loss_grad(xv, wv, grad=gv)
    loss_ref, g_ref = oracle.loss_grad(x.astype(np.complex128), w.astype(np.float64))
    assert per_transform_relerr(gv.cpu().numpy(), g_ref) <= TOL
    assert abs(float(loss.double().sum()) - loss_ref) / loss_ref < 1e-5


def test_below_element_alignment_is_refused():
    """complex64 data at a 4-byte offset, 16-bit pairs at a 2-byte offset:
    FFT_EALIGN from the C ABI, nothing launched."""
    L = native.lib()
    n, batch = 256, 4
    buf = torch.zeros(2 * n * batch + 8, dtype=torch.float32, device="cuda")
    out = torch.empty_like(buf)
    p = api.Plan(n, batch, -1)
    base, obase = buf.data_ptr(), out.data_ptr()
    rc = L.fft_execute(p._h, ctypes.c_void_p(base + 4), ctypes.c_void_p(obase), None)
    assert native.STATUS[rc] == "FFT_EALIGN"
    rc = L.fft_execute(p._h, ctypes.c_void_p(base), ctypes.c_void_p(obase + 12), None)
    assert native.STATUS[rc] == "FFT_EALIGN"
    ph = api.Plan(n, batch, -1, dtype="c16")
    rc = L.fft_execute(ph._h, ctypes.c_void_p(base + 2), ctypes.c_void_p(obase), None)
    assert native.STATUS[rc] == "FFT_EALIGN"
    pr = api.Plan(n, batch, -1, dtype="r32")
    rc = L.fft_execute(pr._h, ctypes.c_void_p(base + 4), ctypes.c_void_p(obase + 4), None)  # bins side 4 B
    assert native.STATUS[rc] == "FFT_EALIGN"
    rc = L.fft_execute(pr._h, ctypes.c_void_p(base + 4), ctypes.c_void_p(obase + 8), None)
    assert rc == 0
    torch.cuda.synchronize()
